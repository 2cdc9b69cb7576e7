"""FP64 CPU oracle for stochastic convolutional sparse coding -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import anything from here.  The product path (the HIP library and its
Python binding) never imports it and shares no code with it.

Pins (all in ``tests/test_oracle_*.py``, run without a GPU):
* synthesis / adjoint / filter correlation: scipy.signal convolve2d and
  correlate2d, the adjoint identities, and brute-force loops on tiny inputs;
* Philox4x32-10: known answers from rocRAND's open-source header compiled on
  the host, plus Bernoulli statistics;
* code step: the delta-filter closed form S_lambda(x) on the sample, the
  lambda >= lambda_max zero solution, monotone objective at p = 1, and the
  converged solution against scikit-learn's coordinate-descent Lasso on the
  explicit subsampled operator;
* step sizes: L_z >= ||D||^2 by SVD of the explicit operator, L_d against
  eigvalsh of the explicit (masked, or zero-padded) normal matrix, the padded
  matrix against brute-force lag sums and its dominance over the exact one;
* filter steps: the single-delta-code closed form, the surrogate identity
  C d - B = -Z^T W r, symmetry / PSD and the eq. (8) recursion.
"""

from .csc import (  # noqa: F401
    OnlineState,
    adjoint,
    bernoulli_mask,
    code_matrix,
    code_step,
    code_step_admm,
    dft_size,
    dict_step_batch,
    dict_step_online,
    filter_corr,
    inpaint,
    lipschitz_code,
    lipschitz_filter,
    normal_matvec,
    pad_codes,
    objective,
    project_ball,
    psnr,
    sample_threshold,
    soft_threshold,
    surrogate_increment,
    synthesize,
)
from .philox import philox4x32_10  # noqa: F401
