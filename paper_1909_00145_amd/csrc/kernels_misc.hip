// FP64 reductions for gfx950: the objective of eq. (1) and the Lipschitz bound
// of the code gradient used as the proximal-gradient step size.
#include "scsc_internal.h"

namespace scsc {

namespace {

template <int NT>
__device__ __forceinline__ double block_sum_d(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    double s = red[0];
    __syncthreads();
    return s;
}

// Objective per tile: the reconstruction is formed in FP64 from the dense codes
// (filter by filter, the code map of the tile grown by c pixels staged in LDS;
// maps that are zero on the whole region are skipped), then
// 1/2 (W (x - D z))^2 and |z| are reduced in FP64 in a fixed order.
template <int MM>
__global__ __launch_bounds__(TPB) void k_objective(const ImgInfo *imgs, const TileInfo *tiles, int K,
                                                   const float *__restrict__ x, const unsigned char *__restrict__ W,
                                                   const float *__restrict__ d, const float *__restrict__ z,
                                                   double *__restrict__ partial) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM;
    __shared__ float zr[RW * RW];
    __shared__ double dk[M];
    __shared__ double red[TPB];
    const TileInfo t = tiles[blockIdx.x];
    const ImgInfo im = imgs[t.img];
    const int ly = threadIdx.x / TS, lx = threadIdx.x % TS;
    const int y = t.ty * TS + ly, xx = t.tx * TS + lx;
    const bool valid = y < im.H && xx < im.W;
    const long long HW = (long long)im.H * im.W;
    const int oy = t.ty * TS - C, ox = t.tx * TS - C;
    double acc = 0.0, l1 = 0.0;
    for (int k = 0; k < K; ++k) {
        const float *zk = z + (long long)K * im.pix_off + (long long)k * HW;
        int any = 0;
        for (int i = threadIdx.x; i < RW * RW; i += TPB) {
            const int gy = oy + i / RW, gx = ox + i % RW;
            float v = 0.f;
            if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) v = zk[(long long)gy * im.W + gx];
            zr[i] = v;
            any |= v != 0.f;
        }
        for (int i = threadIdx.x; i < M; i += TPB) dk[i] = (double)d[(long long)k * M + i];
        if (!__syncthreads_or(any)) continue;
        if (valid) {
            for (int sy = -C; sy <= C; ++sy)
                for (int sx = -C; sx <= C; ++sx)
                    acc += dk[(sy + C) * MM + (sx + C)] * (double)zr[(ly + C - sy) * RW + (lx + C - sx)];
            l1 += fabs((double)zr[(ly + C) * RW + (lx + C)]);
        }
        __syncthreads();
    }
    double data = 0.0;
    if (valid) {
        const long long gp = im.pix_off + (long long)y * im.W + xx;
        double e = (double)x[gp] - acc;
        if (W && !W[gp]) e = 0.0;
        data = 0.5 * e * e;
    }
    data = block_sum_d<TPB>(data, red);
    l1 = block_sum_d<TPB>(l1, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = data;
        partial[2 * blockIdx.x + 1] = l1;
    }
}

__global__ __launch_bounds__(1024) void k_reduce_pairs(const double *partial, int n, double *out) {
    __shared__ double red[1024];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    a = block_sum_d<1024>(a, red);
    b = block_sum_d<1024>(b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// The P roots of unity of the DFT grid: tw[ph] = (cos, sin)(-2 pi ph / P).  Both
// passes index this table with the phase (u b) mod P.
__global__ void k_dft_twiddles(int P, double2 *tw, double *maxv) {
    const int ph = blockIdx.x * blockDim.x + threadIdx.x;
    if (ph == 0) *maxv = 0.0;  // the running maximum of k_dft_max starts from zero
    if (ph >= P) return;
    double sn, cs;
    sincos(-2.0 * M_PI * (double)ph / (double)P, &sn, &cs);
    tw[ph] = make_double2(cs, sn);
}

// Row DFT of every filter row, zero padded to P: F1[k][a][u] = sum_b d[k][a][b] e^{-2 pi i u b / P}.
__global__ void k_dft_rows(const float *d, int K, int m, int P, const double2 *__restrict__ tw, double2 *F1) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)K * m * P;
    if (i >= n) return;
    const int u = (int)(i % P);
    const long long ka = i / P;
    const float *row = d + ka * m;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < m; ++b) {
        const double2 t = tw[((long long)u * b) % P];
        re += (double)row[b] * t.x;
        im += (double)row[b] * t.y;
    }
    F1[i] = make_double2(re, im);
}

// Column DFT and the power sum over a chunk of DFT_KC filters at every
// frequency (v, u): part[chunk][v P + u].
constexpr int DFT_KC = 8;

__global__ __launch_bounds__(256) void k_dft_cols(const double2 *F1, int K, int m, int P,
                                                   const double2 *__restrict__ tw, double *part) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)P * P) return;
    const int u = (int)(i % P), v = (int)(i / P);
    double tc[2 * MAX_C + 1], ts[2 * MAX_C + 1];
#pragma unroll
    for (int a = 0; a < 2 * MAX_C + 1; ++a) {
        tc[a] = 0.0;
        ts[a] = 0.0;
        if (a < m) {
            const double2 t = tw[((long long)v * a) % P];
            tc[a] = t.x;
            ts[a] = t.y;
        }
    }
    const int k0 = blockIdx.y * DFT_KC, k1 = min(K, k0 + DFT_KC);
    double S = 0.0;
    for (int k = k0; k < k1; ++k) {
        double re = 0.0, im = 0.0;
        const double2 *f1 = F1 + (long long)k * m * P + u;
#pragma unroll
        for (int a = 0; a < 2 * MAX_C + 1; ++a) {
            if (a < m) {
                const double2 f = f1[(long long)a * P];
                re += f.x * tc[a] - f.y * ts[a];
                im += f.x * ts[a] + f.y * tc[a];
            }
        }
        S += re * re + im * im;
    }
    part[(long long)blockIdx.y * P * P + i] = S;
}

// Sum of the chunks in order at every frequency, block maximum folded into
// *out through an integer max on the (non-negative) FP64 bit pattern.
__global__ __launch_bounds__(256) void k_dft_max(const double *part, int nch, long long n, unsigned long long *out) {
    __shared__ double red[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double S = 0.0;
    if (i < n)
        for (int c = 0; c < nch; ++c) S += part[(long long)c * n + i];
    red[threadIdx.x] = S;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

template <int MM>
hipError_t objective_impl(const Geometry &g, int K, const float *x, const unsigned char *W, const float *d,
                          const float *z, double *partial, double *out, hipStream_t s) {
    SCSC_LAUNCH(k_objective<MM>, dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, x, W, d, z, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_reduce_pairs, dim3(1), dim3(1024), 0, s, partial, g.n_tiles, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_objective(const Geometry &g, int K, int m, const float *x, const unsigned char *W, const float *d,
                            const float *z, double *partial, double *out, hipStream_t s) {
    switch (m) {
        case 3: return objective_impl<3>(g, K, x, W, d, z, partial, out, s);
        case 5: return objective_impl<5>(g, K, x, W, d, z, partial, out, s);
        case 7: return objective_impl<7>(g, K, x, W, d, z, partial, out, s);
        case 9: return objective_impl<9>(g, K, x, W, d, z, partial, out, s);
        case 11: return objective_impl<11>(g, K, x, W, d, z, partial, out, s);
        default: return hipErrorInvalidValue;
    }
}

long long lipschitz_tmp_elems(int K, int m, int P) {
    return 2LL * K * m * P + (long long)((K + DFT_KC - 1) / DFT_KC) * P * P + 2LL * P + 1;
}

hipError_t launch_lipschitz_code(const float *d, int K, int m, int P, double *tmp, double *out, hipStream_t s) {
    double2 *F1 = reinterpret_cast<double2 *>(tmp);
    const long long n1 = (long long)K * m * P;
    const long long n2 = (long long)P * P;
    const int nch = (K + DFT_KC - 1) / DFT_KC;
    double *part = tmp + 2LL * K * m * P;
    double2 *tw = reinterpret_cast<double2 *>(part + (long long)nch * n2);  // 2P doubles, 16-byte aligned
    SCSC_LAUNCH(k_dft_twiddles, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, tw, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_dft_rows, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, d, K, m, P, tw, F1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    SCSC_LAUNCH(k_dft_cols, dim3((unsigned)((n2 + 255) / 256), nch), dim3(256), 0, s, F1, K, m, P, tw, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    SCSC_LAUNCH(k_dft_max, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, part, nch, n2,
                reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Elementwise kernels of an unrolled proximal-gradient layer (dense codes).
// ---------------------------------------------------------------------------
namespace {
__global__ void k_ista_update(long long n, const float *__restrict__ z, const float *__restrict__ g,
                              const unsigned char *__restrict__ mask, float eta, float thr, float *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float u = fmaf(eta, g[i], z[i]);
        out[i] = mask[i] ? soft_threshold(u, thr) : 0.f;
    }
}

__global__ void k_ista_grad_u(long long n, const float *__restrict__ z, const float *__restrict__ g,
                              const unsigned char *__restrict__ mask, const float *__restrict__ gout, float eta,
                              float thr, float *__restrict__ gu) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float u = fmaf(eta, g[i], z[i]);
        gu[i] = (mask[i] && fabsf(u) > thr) ? gout[i] : 0.f;
    }
}

__global__ void k_axpby(long long n, float a, const float *__restrict__ x, float b, const float *__restrict__ y,
                        float *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

__global__ void k_set2(float *dst, float a, float b) {
    if (threadIdx.x == 0) dst[0] = a;
    if (threadIdx.x == 1) dst[1] = b;
}

unsigned ew_blocks(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}
}  // namespace

hipError_t launch_ista_update(long long n, const float *z, const float *g, const unsigned char *mask, float eta,
                              float thr, float *out, hipStream_t s) {
    SCSC_LAUNCH(k_ista_update, dim3(ew_blocks(n)), dim3(256), 0, s, n, z, g, mask, eta, thr, out);
    return hipGetLastError();
}

hipError_t launch_ista_grad_u(long long n, const float *z, const float *g, const unsigned char *mask,
                              const float *gout, float eta, float thr, float *gu, hipStream_t s) {
    SCSC_LAUNCH(k_ista_grad_u, dim3(ew_blocks(n)), dim3(256), 0, s, n, z, g, mask, gout, eta, thr, gu);
    return hipGetLastError();
}

hipError_t launch_set2(float *dst, float a, float b, hipStream_t s) {
    SCSC_LAUNCH(k_set2, dim3(1), dim3(64), 0, s, dst, a, b);
    return hipGetLastError();
}

// The step and threshold of a code step, and its counter of list entries set
// to zero: dst = {(float)eta, (float)(eta lambda)} with eta = step when step > 0,
// else eta = 1 / L from the device scalar L (the FP64 operations the host would
// do; 0 when L is not positive).
__global__ void k_set_step(float *dst, const double *L, double step, double lambda, unsigned long long *counter) {
    if (threadIdx.x != 0) return;
    double eta = step;
    if (!(step > 0.0)) {
        const double Lv = *L;
        eta = Lv > 0.0 ? 1.0 / Lv : 0.0;
    }
    dst[0] = (float)eta;
    dst[1] = (float)(eta * lambda);
    *counter = 0ull;
}

hipError_t launch_set_step(float *dst, const double *L, double step, double lambda, unsigned long long *counter,
                           hipStream_t s) {
    SCSC_LAUNCH(k_set_step, dim3(1), dim3(64), 0, s, dst, L, step, lambda, counter);
    return hipGetLastError();
}

hipError_t launch_axpby(long long n, float a, const float *x, float b, const float *y, float *out, hipStream_t s) {
    SCSC_LAUNCH(k_axpby, dim3(ew_blocks(n)), dim3(256), 0, s, n, a, x, b, y, out);
    return hipGetLastError();
}

}  // namespace scsc
