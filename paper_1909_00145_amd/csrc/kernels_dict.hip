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
template <int MM, typename ACC, bool FROM_X>
__global__ __launch_bounds__(TPB) void k_filter_corr(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles, int K,
                                                     Lists zl, const float *__restrict__ r,
                                                     const unsigned char *__restrict__ W, ACC *__restrict__ partial,
                                                     int KC) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM;
    __shared__ float rr[RW * RW];
    __shared__ unsigned loff[TPB];
    __shared__ int lc[TPB];
    extern __shared__ double gshm[];
    ACC *Gp = reinterpret_cast<ACC *>(gshm);
    const int k0 = blockIdx.y * KC;
    const int k1 = min(K, k0 + KC);
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) Gp[i] = ACC(0);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();
        const TileInfo t = tiles[tile];
        const ImgInfo im = imgs[t.img];
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
        {
            const int ly = threadIdx.x / TS, lx = threadIdx.x % TS;
            const int y = t.ty * TS + ly, x = t.tx * TS + lx;
            int n = 0;
            unsigned o = 0;
            if (y < im.H && x < im.W) {
                const long long gp = im.pix_off + (long long)y * im.W + x;
                n = zl.cnt[gp];
                o = zl.off[gp];
            }
            lc[threadIdx.x] = n;
            loff[threadIdx.x] = o;
        }
        __syncthreads();
        for (int px = 0; px < TPB; ++px) {
            const int n = lc[px];
            if (n == 0) continue;
            const unsigned o = loff[px];
            const int qy = px / TS, qx = px % TS;
            for (int j = 0; j < n; ++j) {
                const Pair e = zl.pairs[o + j];
                if (e.k < k0 || e.k >= k1 || ((e.k - k0) & 3) != wave) continue;
                const ACC v = (ACC)e.v;
                ACC *row = Gp + (e.k - k0) * M;
                for (int tt = lane; tt < M; tt += 64) {
                    const int sy = tt / MM - C, sx = tt % MM - C;
                    row[tt] += v * (ACC)rr[(qy + C + sy) * RW + (qx + C + sx)];
                }
            }
        }
    }
    __syncthreads();
    ACC *dst = partial + (long long)blockIdx.x * K * M + (long long)k0 * M;
    for (int i = threadIdx.x; i < (k1 - k0) * M; i += TPB) dst[i] = Gp[i];
}

template <typename ACC>
__global__ void k_reduce_partials(const ACC *__restrict__ partial, int nblocks, int n, ACC *__restrict__ out,
                                  int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ACC s = ACC(0);
    for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * n + i];
    out[i] = accumulate ? out[i] + s : s;
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

// ---------------------------------------------------------------------------
// Surrogate C_bar += sum_p W[p] w_p w_p^T, w_p the row of Z at pixel p (eq. 7).
// Lag layout: entry ((k, s), (k2, s2)) sits in block (k, k2) at lag
// delta = s - s2; a pair of non-zero codes (k, q, v), (k2, q2, v2) with
// q2 - q = delta adds v v2 W[q + s] to every s of that lag whose pixel q + s
// lies in the image, a contiguous run of the lag's row-major s rectangle.
// Blocks own tiles of first codes; partner codes come from the tile grown by
// 2c pixels, staged in LDS.  Lanes of a wave cover the s of one pair, so the
// FP64 atomics of a pair hit consecutive addresses.
// ---------------------------------------------------------------------------
constexpr int SUR_CAP = 4096;

__host__ __device__ __forceinline__ int lag_prefix(int a, int m) {
    // sum_{b = -(m-1)}^{a-1} (m - |b|)
    if (a <= 0) return (m + a - 1) * (m + a) / 2;
    return m * (m - 1) / 2 + a * m - a * (a - 1) / 2;
}

template <int MM>
__global__ __launch_bounds__(TPB) void k_surrogate_accumulate(const ImgInfo *imgs, const TileInfo *tiles, int K,
                                                              Lists zl, const unsigned char *__restrict__ W,
                                                              double *__restrict__ Cbar) {
    constexpr int C = MM / 2, RW = TS + 4 * C, R = RW * RW, M = MM * MM, M2 = M * M;
    constexpr int CH = (R + TPB - 1) / TPB;
    __shared__ unsigned lgoff[R];
    __shared__ int lstart[R];
    __shared__ int lcnt[R];
    __shared__ Pair lp[SUR_CAP];
    __shared__ int scratch[TPB];
    const TileInfo t = tiles[blockIdx.x];
    const ImgInfo im = imgs[t.img];
    const int oy = t.ty * TS - 2 * C, ox = t.tx * TS - 2 * C;
    int mysum = 0;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int i = threadIdx.x * CH + j;
        if (i < R) {
            const int gy = oy + i / RW, gx = ox + i % RW;
            int n = 0;
            unsigned o = 0;
            if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) {
                const long long gp = im.pix_off + (long long)gy * im.W + gx;
                n = zl.cnt[gp];
                o = zl.off[gp];
            }
            lcnt[i] = n;
            lgoff[i] = o;
            mysum += n;
        }
    }
    int total;
    int ex = block_exclusive_scan(mysum, scratch, &total);
    const bool staged = total <= SUR_CAP;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int i = threadIdx.x * CH + j;
        if (i < R) {
            lstart[i] = ex;
            if (staged)
                for (int q = 0; q < lcnt[i]; ++q) lp[ex + q] = zl.pairs[lgoff[i] + q];
            ex += lcnt[i];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int e_idx = 0;
    for (int px = 0; px < TPB; ++px) {
        const int ly = px / TS, lx = px % TS;
        const int qy = t.ty * TS + ly, qx = t.tx * TS + lx;
        if (qy >= im.H || qx >= im.W) continue;
        const int ri = (ly + 2 * C) * RW + (lx + 2 * C);
        const int n1 = lcnt[ri];
        for (int a = 0; a < n1; ++a, ++e_idx) {
            if ((e_idx & 3) != wave) continue;
            const Pair e1 = staged ? lp[lstart[ri] + a] : zl.pairs[lgoff[ri] + a];
            for (int dy = -2 * C; dy <= 2 * C; ++dy) {
                const int wy = MM - (dy < 0 ? -dy : dy);
                const int sylo = max(-C, dy - C);
                for (int dx = -2 * C; dx <= 2 * C; ++dx) {
                    const int rj = (ly + 2 * C + dy) * RW + (lx + 2 * C + dx);
                    const int n2 = lcnt[rj];
                    if (n2 == 0) continue;
                    const int wx = MM - (dx < 0 ? -dx : dx);
                    const int sxlo = max(-C, dx - C);
                    const long long lag_off = (long long)lag_prefix(dy, MM) * M + (long long)wy * lag_prefix(dx, MM);
                    const int nrect = wy * wx;
                    for (int b = 0; b < n2; ++b) {
                        const Pair e2 = staged ? lp[lstart[rj] + b] : zl.pairs[lgoff[rj] + b];
                        const double vv = (double)e1.v * (double)e2.v;
                        double *blk = Cbar + ((long long)e1.k * K + e2.k) * M2 + lag_off;
                        for (int ti = lane; ti < nrect; ti += 64) {
                            const int sy = sylo + ti / wx, sx = sxlo + ti % wx;
                            const int py = qy + sy, pxx = qx + sx;
                            if (py < 0 || py >= im.H || pxx < 0 || pxx >= im.W) continue;
                            if (W && !W[im.pix_off + (long long)py * im.W + pxx]) continue;
                            atomicAdd(blk + ti, vv);
                        }
                    }
                }
            }
        }
    }
}

// y = C_bar d in the lag layout.  Block (k, chunk of SMV_KB filters k2),
// thread <-> tap s of row k; for each lag the valid threads read a contiguous
// run of the block.  Partials over k2 chunks are reduced in a fixed order.
constexpr int SMV_KB = 4;

template <int MM>
__global__ __launch_bounds__(128) void k_surrogate_matvec(int K, const double *__restrict__ Cbar,
                                                          const float *__restrict__ d, double *__restrict__ partial) {
    constexpr int C = MM / 2, M = MM * MM, M2 = M * M;
    __shared__ double dl[SMV_KB * M];
    const int k = blockIdx.x;
    const int kc = blockIdx.y;
    const int k2a = kc * SMV_KB, k2b = min(K, k2a + SMV_KB);
    for (int i = threadIdx.x; i < (k2b - k2a) * M; i += 128) dl[i] = (double)d[(long long)k2a * M + i];
    __syncthreads();
    const int tt = threadIdx.x;
    const bool active = tt < M;
    const int sy = active ? tt / MM - C : 0, sx = active ? tt % MM - C : 0;
    double acc = 0.0;
    for (int k2 = k2a; k2 < k2b; ++k2) {
        const double *blk = Cbar + ((long long)k * K + k2) * M2;
        const double *dk = dl + (k2 - k2a) * M;
        long long off = 0;
        for (int dy = -(MM - 1); dy <= MM - 1; ++dy) {
            const int wy = MM - (dy < 0 ? -dy : dy);
            const int sylo = max(-C, dy - C), syhi = min(C, dy + C);
            const bool rowok = active && sy >= sylo && sy <= syhi;
            for (int dx = -(MM - 1); dx <= MM - 1; ++dx) {
                const int wx = MM - (dx < 0 ? -dx : dx);
                const int sxlo = max(-C, dx - C), sxhi = min(C, dx + C);
                if (rowok && sx >= sxlo && sx <= sxhi) {
                    const double c = blk[off + (sy - sylo) * wx + (sx - sxlo)];
                    acc += c * dk[(sy - dy + C) * MM + (sx - dx + C)];
                }
                off += wy * wx;
            }
        }
    }
    if (active) partial[(long long)kc * K * M + (long long)k * M + tt] = acc;
}

template <int MM, typename ACC, bool FROM_X>
hipError_t corr_impl(const Geometry &g, int K, Lists z, const float *r, const unsigned char *W, ACC *partial,
                     int nblocks, hipStream_t s) {
    constexpr int M = MM * MM;
    int KC = (56 * 1024) / (M * (int)sizeof(ACC));
    KC = KC / 4 * 4;
    if (KC > K) KC = K;
    const int nkc = (K + KC - 1) / KC;
    const size_t shm = (size_t)KC * M * sizeof(ACC);
    hipLaunchKernelGGL((k_filter_corr<MM, ACC, FROM_X>), dim3(nblocks, nkc), dim3(TPB), shm, s, g.d_img, g.d_tiles,
                       g.n_tiles, K, z, r, W, partial, KC);
    return hipGetLastError();
}

template <int MM>
hipError_t corr_f32_impl(const Geometry &g, int K, Lists z, const float *r, float *partial, int nblocks,
                         hipStream_t s) {
    return corr_impl<MM, float, false>(g, K, z, r, nullptr, partial, nblocks, s);
}

template <int MM>
hipError_t corr_f64_impl(const Geometry &g, int K, Lists z, const float *x, const unsigned char *W, double *partial,
                         int nblocks, hipStream_t s) {
    return corr_impl<MM, double, true>(g, K, z, x, W, partial, nblocks, s);
}

template <int MM>
hipError_t sur_acc_impl(const Geometry &g, int K, Lists z, const unsigned char *W, double *C, hipStream_t s) {
    hipLaunchKernelGGL(k_surrogate_accumulate<MM>, dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, z, W, C);
    return hipGetLastError();
}

template <int MM>
hipError_t sur_mv_impl(int K, const double *C, const float *d, double *partial, double *y, hipStream_t s) {
    constexpr int M = MM * MM;
    const int nkc = (K + SMV_KB - 1) / SMV_KB;
    hipLaunchKernelGGL(k_surrogate_matvec<MM>, dim3(K, nkc), dim3(128), 0, s, K, C, d, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = K * M;
    hipLaunchKernelGGL(k_reduce_partials<double>, dim3((n + 255) / 256), dim3(256), 0, s, partial, nkc, n, y, 0);
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
    hipLaunchKernelGGL(k_reduce_partials<float>, dim3((n + 255) / 256), dim3(256), 0, s, partial, nblocks, n, out, 0);
    return hipGetLastError();
}

hipError_t launch_reduce_partials_f64_add(const double *partial, int nblocks, int n, double *inout, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials<double>, dim3((n + 255) / 256), dim3(256), 0, s, partial, nblocks, n, inout,
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

hipError_t launch_surrogate_accumulate(const Geometry &g, int K, int m, Lists z, const unsigned char *W, double *C,
                                       hipStream_t s) {
    SCSC_DISPATCH_M(m, sur_acc_impl, g, K, z, W, C, s);
}

long long surrogate_matvec_partial_elems(int K, int m) {
    return (long long)((K + SMV_KB - 1) / SMV_KB) * K * m * m;
}

hipError_t launch_surrogate_matvec(int K, int m, const double *C, const float *d, double *partial, double *y,
                                   hipStream_t s) {
    SCSC_DISPATCH_M(m, sur_mv_impl, K, C, d, partial, y, s);
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
