// Filter correlation G[k][t] = sum_i sum_q z_i,k[q] r_i[q + t] (the filter
// gradient Z^T r of eq. (5)) as an implicit-im2col GEMM on the matrix cores:
// per 16 x 16 pixel tile, M = filters, N = taps, K-dim = the tile's 256 pixels,
// with the codes (scattered from their per-pixel lists into a dense tile) and
// the residual window rounded to BF16 and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Workgroups stride over the tiles, keep their
// sums in registers and write one partial [K][m^2] each; the partials are then
// added in a fixed order in FP64.
#include "scsc_internal.h"

namespace scsc {
namespace {

constexpr int CM_FG = 128;        // filters per workgroup (eight 16-row tiles)
constexpr int CM_ZS = TPB + 8;    // LDS row stride of the code tile (bf16), padded against bank conflicts

template <int MM>
__global__ __launch_bounds__(TPB) void k_corr_mfma(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles, int K,
                                                   Lists zl, const float *__restrict__ r, float *__restrict__ part) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM;
    constexpr int NCT = (M + 15) / 16;       // 16-tap column tiles
    constexpr int NCW = (NCT + 3) / 4;       // column tiles per wave
    __shared__ bf16x8 zt8[CM_FG * CM_ZS / 8];  // [filter][pixel] codes of the tile
    __shared__ __bf16 rb[RW * RW];
    __bf16 *zt = reinterpret_cast<__bf16 *>(zt8);

    const int kg0 = blockIdx.y * CM_FG, nkg = min(CM_FG, K - kg0), nrt = (nkg + 15) >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fcol = lane & 15, fk = 8 * (lane >> 4);
    f32x4 acc[8][NCW];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < NCW; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const PixelCtx c = pixel_ctx(imgs, tiles, tile);
        __syncthreads();  // the previous tile's fragments have been read
        for (int i = threadIdx.x; i < CM_FG * CM_ZS / 8; i += TPB) zt8[i] = bf16x8{};
        const int oy = c.t.ty * TS - C, ox = c.t.tx * TS - C;
        for (int i = threadIdx.x; i < RW * RW; i += TPB) {
            const int gy = oy + i / RW, gx = ox + i % RW;
            float v = 0.f;
            if (gy >= 0 && gy < c.im.H && gx >= 0 && gx < c.im.W) v = r[c.im.pix_off + (long long)gy * c.im.W + gx];
            rb[i] = (__bf16)v;
        }
        __syncthreads();
        if (c.valid) {
            const unsigned o = zl.off[c.gp];
            const int n = zl.cnt[c.gp];
            for (int j = 0; j < n; ++j) {
                const Pair e = zl.pairs[o + j];
                if (e.k >= kg0 && e.k < kg0 + nkg) zt[(e.k - kg0) * CM_ZS + threadIdx.x] = (__bf16)e.v;
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < TPB / 32; ++ks) {
            // B fragment: tap t (column), pixels ks*32 + fk .. + 7 (one tile row, consecutive columns)
            const int q0 = ks * 32 + fk, qy = q0 / TS, qx = q0 % TS;
            bf16x8 bfr[NCW];
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) {
                const int t = (wave * NCW + cw) * 16 + fcol;
                const int rowoff = t < M ? (qy + t / MM) * RW + qx + t % MM : 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) bfr[cw][i] = t < M ? rb[rowoff + i] : (__bf16)0.f;
            }
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) {
                if (rt < nrt) {
                    const bf16x8 a = zt8[((rt * 16 + fcol) * CM_ZS + q0) / 8];
#pragma unroll
                    for (int cw = 0; cw < NCW; ++cw)
                        if ((wave * NCW + cw) < NCT)
                            acc[rt][cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[cw], acc[rt][cw], 0, 0, 0);
                }
            }
        }
    }
    // partial [blockIdx.x][K][M]: rows of this filter group, taps < M
    float *dst = part + (long long)blockIdx.x * K * M;
#pragma unroll
    for (int rt = 0; rt < 8; ++rt) {
        if (rt >= nrt) continue;
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            const int t = (wave * NCW + cw) * 16 + fcol;
            if (t >= M) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kk = rt * 16 + (lane >> 4) * 4 + i;
                if (kk < nkg) dst[(long long)(kg0 + kk) * M + t] = acc[rt][cw][i];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_reduce_f32_partials_f64(const float *__restrict__ part, int nblocks, int n,
                                                                 float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)part[(long long)b * n + i];
    out[i] = (float)s;
}

template <int MM>
hipError_t corr_mfma_impl(const Geometry &g, int K, Lists z, const float *r, float *part, int nblk, float *G,
                          hipStream_t s) {
    const int ngroups = (K + CM_FG - 1) / CM_FG;
    hipLaunchKernelGGL(k_corr_mfma<MM>, dim3(nblk, ngroups), dim3(TPB), 0, s, g.d_img, g.d_tiles, g.n_tiles, K, z,
                       r, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = K * MM * MM;
    hipLaunchKernelGGL(k_reduce_f32_partials_f64, dim3((n + 255) / 256), dim3(256), 0, s, part, nblk, n, G);
    return hipGetLastError();
}

}  // namespace

int corr_mfma_blocks(const Geometry &g, int K) {
    const int ngroups = (K + CM_FG - 1) / CM_FG;
    int nb = 512 / ngroups;
    if (nb < 1) nb = 1;
    return nb < g.n_tiles ? nb : g.n_tiles;
}

hipError_t launch_corr_mfma(const Geometry &g, int K, int m, Lists z, const float *r, float *part, float *G,
                            hipStream_t s) {
    const int nblk = corr_mfma_blocks(g, K);
    switch (m) {
        case 3: return corr_mfma_impl<3>(g, K, z, r, part, nblk, G, s);
        case 5: return corr_mfma_impl<5>(g, K, z, r, part, nblk, G, s);
        case 7: return corr_mfma_impl<7>(g, K, z, r, part, nblk, G, s);
        case 9: return corr_mfma_impl<9>(g, K, z, r, part, nblk, G, s);
        case 11: return corr_mfma_impl<11>(g, K, z, r, part, nblk, G, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace scsc
