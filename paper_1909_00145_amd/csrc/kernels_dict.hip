// Filter-update kernels for gfx950: the filter correlation Z^T r of eq. (5),
// power iteration for its step size, the projected updates, and the online
// surrogates of eqs. (7)-(8) in FP64.
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
// FROM_X selects the right-hand side W x (for B of eq. 7) instead of r.
// ---------------------------------------------------------------------------
constexpr int CORR_CAP = 2048;
constexpr double FIX_SCALE = 1099511627776.0;  // 2^40
constexpr double FIX_INV = 1.0 / 1099511627776.0;

// Stage the "right-hand side" region (r, or W x) and the tile's non-zero codes.
// Returns through the shared arrays; contains block barriers.
template <int MM, bool FROM_X>
__device__ __forceinline__ bool corr_stage_tile(const ImgInfo &im, const TileInfo &t, Lists zl,
                                                const float *__restrict__ r, const unsigned char *__restrict__ W,
                                                float *rr, unsigned *loff, int *lst, int *lc, Pair *ent,
                                                int *scratch) {
    constexpr int C = MM / 2, RW = TS + 2 * C;
    const int oy = t.ty * TS - C, ox = t.tx * TS - C;
    for (int i = threadIdx.x; i < RW * RW; i += TPB) {
        const int gy = oy + i / RW, gx = ox + i % RW;
        float v = 0.f;
        if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) {
            const long long gp = im.pix_off + (long long)gy * im.W + gx;
            v = r[gp];
            if (FROM_X && W && !W[gp]) v = 0.f;
        }
        rr[i] = v;
    }
    int n = 0;
    unsigned o = 0;
    {
        const int ly = threadIdx.x / TS, lx = threadIdx.x % TS;
        const int y = t.ty * TS + ly, x = t.tx * TS + lx;
        if (y < im.H && x < im.W) {
            const long long gp = im.pix_off + (long long)y * im.W + x;
            n = zl.cnt[gp];
            o = zl.off[gp];
        }
    }
    int total;
    const int ex = block_exclusive_scan(n, scratch, &total);
    const bool staged = total <= CORR_CAP;
    lc[threadIdx.x] = n;
    loff[threadIdx.x] = o;
    lst[threadIdx.x] = ex;
    if (staged)
        for (int j = 0; j < n; ++j) ent[ex + j] = zl.pairs[o + j];
    __syncthreads();
    return staged;
}

// FP32 filter correlation G_k[s] = sum_q z_k[q] r[q + s].  Each block owns a
// fixed, strided set of tiles and a chunk of filters.  Waves take whole codes,
// lanes the taps; the exact FP64 product of two floats is rounded to a 2^-40
// fixed-point grid and added with an integer LDS atomic, so the block partial
// does not depend on the order of the additions (deterministic).
template <int MM>
__global__ __launch_bounds__(TPB) void k_filter_corr_fix(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles,
                                                         int K, Lists zl, const float *__restrict__ r,
                                                         float *__restrict__ partial, int KC) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM;
    __shared__ float rr[RW * RW];
    __shared__ unsigned loff[TPB];
    __shared__ int lst[TPB];
    __shared__ int lc[TPB];
    __shared__ Pair ent[CORR_CAP];
    __shared__ int scratch[TPB];
    extern __shared__ double gshm[];
    unsigned long long *Gp = reinterpret_cast<unsigned long long *>(gshm);
    const int k0 = blockIdx.y * KC;
    const int k1 = min(K, k0 + KC);
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) Gp[i] = 0ull;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();
        const TileInfo t = tiles[tile];
        const ImgInfo im = imgs[t.img];
        const bool staged = corr_stage_tile<MM, false>(im, t, zl, r, nullptr, rr, loff, lst, lc, ent, scratch);
        if (staged) {
            // flat walk over the tile's codes; pixel of code e from the prefix lst
            int px = 0;
            const int total = lst[TPB - 1] + lc[TPB - 1];
            for (int e = wave; e < total; e += TPB / 64) {
                while (px + 1 < TPB && lst[px + 1] <= e) ++px;
                const Pair en = ent[e];
                if (en.k < k0 || en.k >= k1) continue;
                const int qy = px / TS, qx = px % TS;
                const double v = (double)en.v;
                unsigned long long *row = Gp + (en.k - k0) * M;
                for (int tt = lane; tt < M; tt += 64) {
                    const int sy = tt / MM - C, sx = tt % MM - C;
                    const double prod = v * (double)rr[(qy + C + sy) * RW + (qx + C + sx)];
                    atomicAdd(row + tt, (unsigned long long)__double2ll_rn(prod * FIX_SCALE));
                }
            }
        } else {
            for (int px = wave; px < TPB; px += TPB / 64) {
                const int cnt = lc[px];
                const int qy = px / TS, qx = px % TS;
                for (int j = 0; j < cnt; ++j) {
                    const Pair en = zl.pairs[loff[px] + j];
                    if (en.k < k0 || en.k >= k1) continue;
                    const double v = (double)en.v;
                    unsigned long long *row = Gp + (en.k - k0) * M;
                    for (int tt = lane; tt < M; tt += 64) {
                        const int sy = tt / MM - C, sx = tt % MM - C;
                        const double prod = v * (double)rr[(qy + C + sy) * RW + (qx + C + sx)];
                        atomicAdd(row + tt, (unsigned long long)__double2ll_rn(prod * FIX_SCALE));
                    }
                }
            }
        }
    }
    __syncthreads();
    float *dst = partial + (long long)blockIdx.x * K * M + (long long)k0 * M;
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) dst[i] = (float)((double)(long long)Gp[i] * FIX_INV);
}

// FP64 correlation with the observation-weighted image, Z^T (W x) for B of
// eq. (7).  Wave w owns the filters k with (k - k0) % 4 == w and lane l the taps
// l, l + 64, so every partial cell has one writer and a fixed order.
template <int MM>
__global__ __launch_bounds__(TPB) void k_filter_corr_x64(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles,
                                                         int K, Lists zl, const float *__restrict__ x,
                                                         const unsigned char *__restrict__ W,
                                                         double *__restrict__ partial, int KC) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM;
    __shared__ float rr[RW * RW];
    __shared__ unsigned loff[TPB];
    __shared__ int lst[TPB];
    __shared__ int lc[TPB];
    __shared__ Pair ent[CORR_CAP];
    __shared__ int scratch[TPB];
    extern __shared__ double gshm[];
    double *Gp = gshm;
    const int k0 = blockIdx.y * KC;
    const int k1 = min(K, k0 + KC);
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) Gp[i] = 0.0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();
        const TileInfo t = tiles[tile];
        const ImgInfo im = imgs[t.img];
        const bool staged = corr_stage_tile<MM, true>(im, t, zl, x, W, rr, loff, lst, lc, ent, scratch);
        for (int px = 0; px < TPB; ++px) {
            const int cnt = lc[px];
            if (cnt == 0) continue;
            const int qy = px / TS, qx = px % TS;
            for (int j = 0; j < cnt; ++j) {
                const Pair e = staged ? ent[lst[px] + j] : zl.pairs[loff[px] + j];
                if (e.k < k0 || e.k >= k1 || ((e.k - k0) & 3) != wave) continue;
                const double v = (double)e.v;
                double *row = Gp + (e.k - k0) * M;
                for (int tt = lane; tt < M; tt += 64) {
                    const int sy = tt / MM - C, sx = tt % MM - C;
                    row[tt] += v * (double)rr[(qy + C + sy) * RW + (qx + C + sx)];
                }
            }
        }
    }
    __syncthreads();
    double *dst = partial + (long long)blockIdx.x * K * M + (long long)k0 * M;
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) dst[i] = Gp[i];
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
hipError_t corr_f32_impl(const Geometry &g, int K, Lists z, const float *r, float *partial, int nblocks,
                         hipStream_t s) {
    constexpr int M = MM * MM;
    int KC = (96 * 1024) / (M * 8);
    if (KC > K) KC = K;
    const int nkc = (K + KC - 1) / KC;
    const size_t shm = (size_t)KC * M * 8;
    hipLaunchKernelGGL(k_filter_corr_fix<MM>, dim3(nblocks, nkc), dim3(TPB), shm, s, g.d_img, g.d_tiles, g.n_tiles,
                       K, z, r, partial, KC);
    return hipGetLastError();
}

template <int MM>
hipError_t corr_f64_impl(const Geometry &g, int K, Lists z, const float *x, const unsigned char *W, double *partial,
                         int nblocks, hipStream_t s) {
    constexpr int M = MM * MM;
    int KC = (96 * 1024) / (M * 8);
    KC = KC / 4 * 4;
    if (KC > K) KC = K;
    const int nkc = (K + KC - 1) / KC;
    const size_t shm = (size_t)KC * M * 8;
    hipLaunchKernelGGL(k_filter_corr_x64<MM>, dim3(nblocks, nkc), dim3(TPB), shm, s, g.d_img, g.d_tiles, g.n_tiles,
                       K, z, x, W, partial, KC);
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

int corr_blocks(const Geometry &g) { return g.n_tiles < CORR_MAX_BLOCKS ? g.n_tiles : CORR_MAX_BLOCKS; }

hipError_t launch_filter_corr_f32(const Geometry &g, int K, int m, Lists z, const float *r, float *partial,
                                  int nblocks, hipStream_t s) {
    SCSC_DISPATCH_M(m, corr_f32_impl, g, K, z, r, partial, nblocks, s);
}

hipError_t launch_filter_corr_f64(const Geometry &g, int K, int m, Lists z, const float *x, const unsigned char *W,
                                  double *partial, int nblocks, hipStream_t s) {
    SCSC_DISPATCH_M(m, corr_f64_impl, g, K, z, x, W, partial, nblocks, s);
}

hipError_t launch_reduce_partials_f32(const float *partial, int nblocks, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials<float>, dim3((n + 15) / 16), dim3(256), 0, s, partial, nblocks, n, out, 0);
    return hipGetLastError();
}

hipError_t launch_reduce_partials_f64_add(const double *partial, int nblocks, int n, double *inout, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials<double>, dim3((n + 15) / 16), dim3(256), 0, s, partial, nblocks, n, inout,
                       1);
    return hipGetLastError();
}

hipError_t launch_fill(float *v, int n, float val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, v, n, val);
    return hipGetLastError();
}

hipError_t launch_power_update(float *v, const float *w, int n, double *lam, hipStream_t s) {
    hipLaunchKernelGGL(k_power_update, dim3(1), dim3(1024), 0, s, v, w, n, lam);
    return hipGetLastError();
}

hipError_t launch_batch_update(float *d, const float *G, const double *lam, int K, int M, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_update, dim3(K), dim3(128), 0, s, d, G, lam, M);
    return hipGetLastError();
}

hipError_t launch_online_update(float *d, const double *y, const double *B, double Ld_sum, int K, int M,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_online_update, dim3(K), dim3(128), 0, s, d, y, B, Ld_sum, M);
    return hipGetLastError();
}

}  // namespace scsc

extern "C" int64_t csc_surrogate_size(int K, int m) {
    if (K < 1 || m < 1) return -1;
    const int64_t M = (int64_t)m * m;
    return (int64_t)K * K * M * M;
}

extern "C" int64_t csc_surrogate_index(int K, int m, int k, int sy, int sx, int k2, int sy2, int sx2) {
    if (K < 1 || m < 1 || (m & 1) == 0) return -1;
    const int c = m / 2;
    if (k < 0 || k >= K || k2 < 0 || k2 >= K) return -1;
    if (sy < -c || sy > c || sx < -c || sx > c || sy2 < -c || sy2 > c || sx2 < -c || sx2 > c) return -1;
    const int dy = sy - sy2, dx = sx - sx2;
    const int64_t M = (int64_t)m * m;
    const int wy = m - (dy < 0 ? -dy : dy), wx = m - (dx < 0 ? -dx : dx);
    const int sylo = dy - c > -c ? dy - c : -c;
    const int sxlo = dx - c > -c ? dx - c : -c;
    const int64_t off = (int64_t)scsc::lag_prefix(dy, m) * M + (int64_t)wy * scsc::lag_prefix(dx, m);
    return ((int64_t)k * K + k2) * M * M + off + (int64_t)(sy - sylo) * wx + (sx - sxlo);
}
