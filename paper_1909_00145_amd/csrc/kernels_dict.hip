// Filter-update kernels for gfx950: the filter correlation Z^T r of eq. (5),
// power iteration for its step size, the projected updates, and the online
// surrogates of eqs. (8)-(9) in FP64.
#include "scsc_internal.h"

namespace scsc {

namespace {

constexpr int CORR_MAX_BLOCKS = 512;

// ---------------------------------------------------------------------------
// Filter correlation G_k[s] = sum_q z_k[q] r[q + s] over the non-zero codes.
// Each block owns a fixed, strided set of tiles and a chunk of filters; its
// partial G lives in LDS.  Wave w of the block owns the filters k with
// (k - k0) % 4 == w and lane l the taps l, l + 64, so every partial cell has a
// single writer and a fixed accumulation order: the result is deterministic.
// FROM_X selects the right-hand side W x (for B of eq. 8) instead of r.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Filter correlation G_k[s] = sum_q z_k[q] r[q + s] (r zero outside the image),
// filter-major: workgroup (chunk c, filter k), thread t <-> tap s.  Every thread
// walks the same codes of filter k (a contiguous range of the per-filter list,
// uniform loads) in list order and accumulates v * r[q + s] in FP64, so the
// result is deterministic and needs no atomics.  weight_rhs multiplies the
// right-hand side by the observation mask (for Z^T W x).
// ---------------------------------------------------------------------------
constexpr int CORR_TARGET_BLOCKS = 4096;

template <int MM>
__global__ __launch_bounds__(128) void k_corr_fm(const ImgInfo *imgs, int K, int R, const unsigned *__restrict__ fm_off,
                                                 const FmCode *__restrict__ fm, const float *__restrict__ r,
                                                 const unsigned char *__restrict__ W, int weight_rhs,
                                                 double *__restrict__ partial) {
    constexpr int C = MM / 2, M = MM * MM;
    const int k = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
    const unsigned a = fm_off[(long long)k * R], b = fm_off[(long long)k * R + R];
    const unsigned n = b - a;
    const unsigned e0 = a + (unsigned)(((unsigned long long)n * ch) / nch);
    const unsigned e1 = a + (unsigned)(((unsigned long long)n * (ch + 1)) / nch);
    const int t = threadIdx.x;
    const bool active = t < M;
    const int sy = active ? t / MM - C : 0, sx = active ? t % MM - C : 0;
    constexpr int U = 4;
    double acc[U] = {0.0, 0.0, 0.0, 0.0};
    for (unsigned e = e0; e < e1; e += U) {
        FmCode c[U];
        float rv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = (e + u < e1) ? fm[e + u] : FmCode{0u, 0.f, 0, 0};
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const ImgInfo im = imgs[c[u].img];
            const int y = (int)(c[u].yx >> 16) + sy, x = (int)(c[u].yx & 0xFFFFu) + sx;
            rv[u] = 0.f;
            if (active && e + u < e1 && y >= 0 && y < im.H && x >= 0 && x < im.W) {
                const long long gp = im.pix_off + (long long)y * im.W + x;
                rv[u] = (weight_rhs && W && !W[gp]) ? 0.f : r[gp];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += (double)c[u].v * (double)rv[u];
    }
    if (active) partial[((long long)ch * K + k) * M + t] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// out[i] (+)= sum_b partial[b][i]: blocks of 16 elements x 16 slices; slice j
// sums the partials b = j, j + 16, ... and the 16 slice sums are added in a
// fixed order, so the result is deterministic.
template <typename ACC>
__global__ __launch_bounds__(256) void k_reduce_partials(const ACC *__restrict__ partial, int nblocks, int n,
                                                         ACC *__restrict__ out, int accumulate) {
    __shared__ ACC red[16][17];
    const int e = threadIdx.x & 15, slice = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + e;
    ACC s = ACC(0);
    if (i < n)
        for (int b = slice; b < nblocks; b += 16) s += partial[(long long)b * n + i];
    red[slice][e] = s;
    __syncthreads();
    if (slice == 0 && i < n) {
        ACC t = ACC(0);
        for (int j = 0; j < 16; ++j) t += red[j][e];
        out[i] = accumulate ? out[i] + t : t;
    }
}

__global__ void k_fill(float *v, int n, float val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
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

// lam = <v, w>; v <- w / ||w|| (FP64 reductions, one block).
__global__ __launch_bounds__(1024) void k_power_update(float *v, const float *w, int n, double *lam) {
    __shared__ double red[1024];
    double dot = 0.0, nn = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double a = v[i], b = w[i];
        dot += a * b;
        nn += b * b;
    }
    dot = block_sum<1024>(dot, red);
    nn = block_sum<1024>(nn, red);
    if (nn > 0.0) {
        const double inv = 1.0 / sqrt(nn);
        for (int i = threadIdx.x; i < n; i += 1024) v[i] = (float)((double)w[i] * inv);
    }
    if (threadIdx.x == 0) *lam = nn > 0.0 ? dot : 0.0;
}

// d_k <- P(d_k + G_k / lam): one block per filter, 128 threads (M <= 121).
// G == nullptr or lam <= 0 leaves only the projection.
__global__ __launch_bounds__(128) void k_batch_update(float *d, const float *G, const double *lam, int M) {
    __shared__ double red[128];
    const int k = blockIdx.x;
    const double L = *lam;
    const double step = L > 0.0 ? 1.0 / L : 0.0;
    double v = 0.0;
    if (threadIdx.x < M) {
        v = (double)d[k * M + threadIdx.x];
        if (G) v += step * (double)G[k * M + threadIdx.x];
    }
    const double n2 = block_sum<128>(v * v, red);
    const double nrm = sqrt(n2);
    if (threadIdx.x < M) d[k * M + threadIdx.x] = (float)(nrm > 1.0 ? v / nrm : v);
}

// d_k <- P(d_k - (y_k - B_k) / Ld_sum).
__global__ __launch_bounds__(128) void k_online_update(float *d, const double *y, const double *B, double Ld_sum,
                                                       int M) {
    __shared__ double red[128];
    const int k = blockIdx.x;
    double v = 0.0;
    if (threadIdx.x < M) {
        const int i = k * M + threadIdx.x;
        v = (double)d[i] - (y[i] - B[i]) / Ld_sum;
    }
    const double n2 = block_sum<128>(v * v, red);
    const double nrm = sqrt(n2);
    if (threadIdx.x < M) d[k * M + threadIdx.x] = (float)(nrm > 1.0 ? v / nrm : v);
}

__host__ __device__ __forceinline__ int lag_prefix(int a, int m) {
    // sum_{b = -(m-1)}^{a-1} (m - |b|)
    if (a <= 0) return (m + a - 1) * (m + a) / 2;
    return m * (m - 1) / 2 + a * m - a * (a - 1) / 2;
}

template <int MM>
hipError_t corr_fm_impl(const Geometry &g, int K, const unsigned *fm_off, const FmCode *fm, const float *r,
                        const unsigned char *W, bool weight_rhs, double *partial, hipStream_t s) {
    SCSC_LAUNCH(k_corr_fm<MM>, dim3(corr_chunks(K), K), dim3(128), 0, s, g.d_img, K, g.n_rows, fm_off, fm, r, W,
                weight_rhs ? 1 : 0, partial);
    return hipGetLastError();
}

}  // namespace

#define SCSC_DISPATCH_M(m, FN, ...)          \
    switch (m) {                             \
        case 3: return FN<3>(__VA_ARGS__);   \
        case 5: return FN<5>(__VA_ARGS__);   \
        case 7: return FN<7>(__VA_ARGS__);   \
        case 9: return FN<9>(__VA_ARGS__);   \
        case 11: return FN<11>(__VA_ARGS__); \
        default: return hipErrorInvalidValue; \
    }

int corr_chunks(int K) {
    int c = (CORR_TARGET_BLOCKS + K - 1) / K;
    return c < 1 ? 1 : (c > 64 ? 64 : c);
}

hipError_t launch_corr_fm(const Geometry &g, int K, int m, const unsigned *fm_off, const FmCode *fm, const float *r,
                          const unsigned char *W, bool weight_rhs, double *partial, hipStream_t s) {
    SCSC_DISPATCH_M(m, corr_fm_impl, g, K, fm_off, fm, r, W, weight_rhs, partial, s);
}

namespace {
__global__ __launch_bounds__(256) void k_reduce_f64_to_f32(const double *__restrict__ partial, int nblocks, int n,
                                                          float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * n + i];
    out[i] = (float)s;
}
}  // namespace

hipError_t launch_reduce_partials_f64_to_f32(const double *partial, int nblocks, int n, float *out, hipStream_t s) {
    SCSC_LAUNCH(k_reduce_f64_to_f32, dim3((n + 255) / 256), dim3(256), 0, s, partial, nblocks, n, out);
    return hipGetLastError();
}

hipError_t launch_reduce_partials_f64_add(const double *partial, int nblocks, int n, double *inout, hipStream_t s) {
    SCSC_LAUNCH(k_reduce_partials<double>, dim3((n + 15) / 16), dim3(256), 0, s, partial, nblocks, n, inout,
                1);
    return hipGetLastError();
}

hipError_t launch_fill(float *v, int n, float val, hipStream_t s) {
    SCSC_LAUNCH(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, v, n, val);
    return hipGetLastError();
}

hipError_t launch_power_update(float *v, const float *w, int n, double *lam, hipStream_t s) {
    SCSC_LAUNCH(k_power_update, dim3(1), dim3(1024), 0, s, v, w, n, lam);
    return hipGetLastError();
}

hipError_t launch_batch_update(float *d, const float *G, const double *lam, int K, int M, hipStream_t s) {
    SCSC_LAUNCH(k_batch_update, dim3(K), dim3(128), 0, s, d, G, lam, M);
    return hipGetLastError();
}

hipError_t launch_online_update(float *d, const double *y, const double *B, double Ld_sum, int K, int M,
                                hipStream_t s) {
    SCSC_LAUNCH(k_online_update, dim3(K), dim3(128), 0, s, d, y, B, Ld_sum, M);
    return hipGetLastError();
}

}  // namespace scsc

extern "C" int64_t csc_surrogate_size(int K, int m) {
    if (K < 1 || m < 1) return -1;
    const int64_t M = (int64_t)m * m;
    return (int64_t)K * (K + 1) / 2 * M * M;
}

extern "C" int64_t csc_surrogate_index(int K, int m, int k, int sy, int sx, int k2, int sy2, int sx2) {
    if (K < 1 || m < 1 || (m & 1) == 0) return -1;
    const int c = m / 2;
    if (k < 0 || k >= K || k2 < 0 || k2 >= K) return -1;
    if (sy < -c || sy > c || sx < -c || sx > c || sy2 < -c || sy2 > c || sx2 < -c || sx2 > c) return -1;
    if (k > k2) {  // stored as the transposed entry of block (k2, k)
        int t = k;
        k = k2;
        k2 = t;
        t = sy;
        sy = sy2;
        sy2 = t;
        t = sx;
        sx = sx2;
        sx2 = t;
    }
    const int dy = sy - sy2, dx = sx - sx2;
    const int64_t M = (int64_t)m * m;
    const int wy = m - (dy < 0 ? -dy : dy), wx = m - (dx < 0 ? -dx : dx);
    const int sylo = dy - c > -c ? dy - c : -c;
    const int sxlo = dx - c > -c ? dx - c : -c;
    const int64_t off = (int64_t)scsc::lag_prefix(dy, m) * M + (int64_t)wy * scsc::lag_prefix(dx, m);
    return scsc::tri_block(k, k2, K) * M * M + off + (int64_t)(sy - sylo) * wx + (sx - sxlo);
}
