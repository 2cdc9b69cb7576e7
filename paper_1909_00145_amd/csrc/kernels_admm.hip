// The paper's ADMM code solver (Sec. 3.2, the paragraph after Alg. 1) on the
// sample S: vectors over the selected coordinates ("S-vectors", FP32, nsel
// entries in pixel-major order, each pixel's selected filters ascending at
// [soff[p], soff[p + 1])), the quadratic substep by conjugate gradient with its
// scalars kept in device memory, and the shrinkage / dual update.  Alg. 1 solves
// the code problem of every image on its own, so the CG scalars are per image:
// image n owns the entries [seg[n], seg[n + 1]) and the dot products and CG
// updates run over those segments.
#include "scsc_internal.h"

namespace scsc {
namespace {

constexpr int AD_BLOCKS = 64;  // workgroups per image for the segmented dot products and CG updates

// Every selected coordinate of every pixel as a list entry (k, z_prev[k]), and
// the per-pixel selected counts: the S-vector layout with its filter indices.
__global__ __launch_bounds__(TPB) void k_sel_list(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                  const unsigned *mask_words, const unsigned *soff, const float *z,
                                                  Pair *pairs, unsigned short *cnt) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = soff[c.gp];
    int nn = 0;
    unsigned bits = 0;
    for (int k = 0; k < K; ++k) {
        if ((k & 31) == 0) bits = mask_words[(long long)(k >> 5) * n_pix + c.gp];
        if ((bits >> (k & 31)) & 1u) pairs[base + nn++] = Pair{k, zp[(long long)k * HW]};
    }
    cnt[c.gp] = (unsigned short)nn;
}

// pairs[j] = (sel[j].k, val[j]), or (sel[j].k, sel[j].v) when val is null.
__global__ void k_pack(const Pair *sel, const float *val, Pair *pairs, long long n) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
        pairs[j] = Pair{sel[j].k, val ? val[j] : sel[j].v};
}

// S-vector of a compact list (the non-zero entries of some of a pixel's selected
// filters, ascending): out[j] = the entry's value for selected filter sel[j].k, 0 if absent.
__global__ __launch_bounds__(TPB) void k_unpack(const ImgInfo *imgs, int n_img, long long n_pix,
                                                const unsigned *soff, const Pair *sel, const Pair *cl,
                                                const unsigned short *ccnt, float *out) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const unsigned b = soff[c.gp], e = soff[c.gp + 1];
    const int n = ccnt[c.gp];
    int i = 0;
    Pair ce = n > 0 ? cl[b] : Pair{INT_MAX, 0.f};
    for (unsigned j = b; j < e; ++j) {
        const int k = sel[j].k;
        float v = 0.f;
        if (ce.k == k) {
            v = ce.v;
            ++i;
            ce = i < n ? cl[b + i] : Pair{INT_MAX, 0.f};
        }
        out[j] = v;
    }
}

// Segment starts: seg[n] = soff[first pixel of image n], seg[n_img] = soff[n_pix].
__global__ void k_seg(const ImgInfo *imgs, int n_img, long long n_pix, const unsigned *soff, unsigned *seg) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n <= n_img; n += gridDim.x * blockDim.x)
        seg[n] = soff[n < n_img ? imgs[n].pix_off : n_pix];
}

// part[n][block] = sum over workgroup blockIdx.x's slice of image n's segment of a[j] * b[j], FP64.
__global__ __launch_bounds__(256) void k_dot_part(const float *a, const float *b, const unsigned *seg, double *part) {
    __shared__ double red[256];
    const unsigned lo = seg[blockIdx.y], hi = seg[blockIdx.y + 1];
    double s = 0.0;
    for (unsigned j = lo + blockIdx.x * 256 + threadIdx.x; j < hi; j += gridDim.x * 256)
        s += (double)a[j] * (double)b[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// The CG scalars, in fixed order from the partials of one dot product:
//   mode 0: rr = sum                  (after r is formed)
//   mode 1: alpha = rr / sum          (sum = q . Aq; alpha = 0 when rr or sum is 0)
//   mode 2: beta = sum / rr, rr = sum (sum = the new r . r; beta = 0 when rr is 0)
// sc[n] = {rr, alpha, beta} as doubles for image n (thread n).
__global__ void k_cg_scalar(const double *part, int nb, int n_img, int mode, double *scs) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_img) return;
    double *sc = scs + 3LL * n;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[(long long)n * nb + i];
    if (mode == 0) {
        sc[0] = s;
    } else if (mode == 1) {
        sc[1] = (sc[0] > 0.0 && s > 0.0) ? sc[0] / s : 0.0;
    } else {
        sc[2] = sc[0] > 0.0 ? s / sc[0] : 0.0;
        sc[0] = s;
    }
}

// y += sgn * alpha_n * x over image n = blockIdx.y's segment
__global__ void k_axpy_alpha(float *y, const float *x, const double *scs, const unsigned *seg, float sgn) {
    const float a = sgn * (float)scs[3LL * blockIdx.y + 1];
    const unsigned lo = seg[blockIdx.y], hi = seg[blockIdx.y + 1];
    for (unsigned j = lo + blockIdx.x * blockDim.x + threadIdx.x; j < hi; j += gridDim.x * blockDim.x)
        y[j] = fmaf(a, x[j], y[j]);
}

// q = r + beta_n q over image n = blockIdx.y's segment
__global__ void k_cg_dir(float *q, const float *r, const double *scs, const unsigned *seg) {
    const float b = (float)scs[3LL * blockIdx.y + 2];
    const unsigned lo = seg[blockIdx.y], hi = seg[blockIdx.y + 1];
    for (unsigned j = lo + blockIdx.x * blockDim.x + threadIdx.x; j < hi; j += gridDim.x * blockDim.x)
        q[j] = fmaf(b, q[j], r[j]);
}

// Aq += rho q   (the + rho I of the quadratic substep)
__global__ void k_add_scaled(float *Aq, const float *q, float rho, long long n) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
        Aq[j] = fmaf(rho, q[j], Aq[j]);
}

// r = b0 + rho (v - u) - Aq,  q = r   (the right-hand side minus the operator at the warm start)
__global__ void k_cg_init(float *r, float *q, const float *b0, const float *v, const float *u, const float *Aq,
                          float rho, long long n) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
        const float t = fmaf(rho, v[j] - u[j], b0[j]) - Aq[j];
        r[j] = t;
        q[j] = t;
    }
}

// zh = alpha zt + (1 - alpha) v;  v = S_thr(zh + u);  u = u + zh - v
__global__ void k_admm_update(const float *zt, float *v, float *u, float alpha, float thr, long long n) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
        const float zh = fmaf(alpha, zt[j], (1.f - alpha) * v[j]);
        const float w = zh + u[j];
        const float a = fabsf(w) - thr;
        const float vn = a > 0.f ? copysignf(a, w) : 0.f;
        v[j] = vn;
        u[j] = u[j] + zh - vn;
    }
}

inline unsigned vec_grid(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_sel_list(const Geometry &g, int K, const unsigned *mask_words, const unsigned *soff, const float *z,
                           Pair *pairs, unsigned short *cnt, hipStream_t s) {
    SCSC_LAUNCH(k_sel_list, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K,
                mask_words, soff, z, pairs, cnt);
    return hipGetLastError();
}

hipError_t launch_pack(const Pair *sel, const float *val, Pair *pairs, long long n, hipStream_t s) {
    SCSC_LAUNCH(k_pack, dim3(vec_grid(n)), dim3(256), 0, s, sel, val, pairs, n);
    return hipGetLastError();
}

hipError_t launch_unpack(const Geometry &g, const unsigned *soff, const Pair *sel, const Pair *cl,
                         const unsigned short *ccnt, float *out, hipStream_t s) {
    SCSC_LAUNCH(k_unpack, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, soff, sel, cl,
                ccnt, out);
    return hipGetLastError();
}

long long admm_dot_elems(int n_img) { return (long long)AD_BLOCKS * n_img; }

hipError_t launch_seg(const Geometry &g, const unsigned *soff, unsigned *seg, hipStream_t s) {
    SCSC_LAUNCH(k_seg, dim3((g.n_img + 256) / 256), dim3(256), 0, s, g.d_img, g.n_img, g.n_pix, soff, seg);
    return hipGetLastError();
}

hipError_t launch_cg_dot(const Geometry &g, const float *a, const float *b, const unsigned *seg, double *part,
                         int mode, double *scs, hipStream_t s) {
    SCSC_LAUNCH(k_dot_part, dim3(AD_BLOCKS, g.n_img), dim3(256), 0, s, a, b, seg, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_cg_scalar, dim3((g.n_img + 63) / 64), dim3(64), 0, s, part, AD_BLOCKS, g.n_img, mode, scs);
    return hipGetLastError();
}

hipError_t launch_axpy_alpha(const Geometry &g, float *y, const float *x, const double *scs, const unsigned *seg,
                             float sgn, hipStream_t s) {
    SCSC_LAUNCH(k_axpy_alpha, dim3(AD_BLOCKS, g.n_img), dim3(256), 0, s, y, x, scs, seg, sgn);
    return hipGetLastError();
}

hipError_t launch_cg_dir(const Geometry &g, float *q, const float *r, const double *scs, const unsigned *seg,
                         hipStream_t s) {
    SCSC_LAUNCH(k_cg_dir, dim3(AD_BLOCKS, g.n_img), dim3(256), 0, s, q, r, scs, seg);
    return hipGetLastError();
}

hipError_t launch_add_scaled(float *Aq, const float *q, float rho, long long n, hipStream_t s) {
    SCSC_LAUNCH(k_add_scaled, dim3(vec_grid(n)), dim3(256), 0, s, Aq, q, rho, n);
    return hipGetLastError();
}

hipError_t launch_cg_init(float *r, float *q, const float *b0, const float *v, const float *u, const float *Aq,
                          float rho, long long n, hipStream_t s) {
    SCSC_LAUNCH(k_cg_init, dim3(vec_grid(n)), dim3(256), 0, s, r, q, b0, v, u, Aq, rho, n);
    return hipGetLastError();
}

hipError_t launch_admm_update(const float *zt, float *v, float *u, float alpha, float thr, long long n,
                              hipStream_t s) {
    SCSC_LAUNCH(k_admm_update, dim3(vec_grid(n)), dim3(256), 0, s, zt, v, u, alpha, thr, n);
    return hipGetLastError();
}

}  // namespace scsc

namespace scsc {
namespace {
__global__ __launch_bounds__(256) void k_count_nz(const float *v, long long n, unsigned long long *out) {
    __shared__ unsigned long long red[256];
    unsigned long long c = 0;
    for (long long j = (long long)blockIdx.x * 256 + threadIdx.x; j < n; j += (long long)gridDim.x * 256)
        c += v[j] != 0.f;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(out, red[0]);
}
}  // namespace

hipError_t launch_count_nz(const float *v, long long n, unsigned long long *out, hipStream_t s) {
    SCSC_LAUNCH(k_count_nz, dim3(vec_grid(n)), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}
}  // namespace scsc
