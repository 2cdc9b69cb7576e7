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

// out[i] = sum_b part[b][i] in FP64: blocks of 16 elements x 16 slices; slice j adds
// the partials b = j, j + 16, ... in order and the 16 slice sums are then added in
// order, so the result is deterministic with 16 times the parallelism of one thread
// per element (one workgroup per tile leaves hundreds of partials).
__global__ __launch_bounds__(256) void k_reduce_f32_partials_f64(const float *__restrict__ part, int nblocks, int n,
                                                                 float *__restrict__ out) {
    __shared__ double red[16][17];
    const int e = threadIdx.x & 15, slice = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + e;
    double s = 0.0;
    if (i < n)
#pragma unroll 4
        for (int b = slice; b < nblocks; b += 16) s += (double)part[(long long)b * n + i];
    red[slice][e] = s;
    __syncthreads();
    if (slice == 0 && i < n) {
        double t = 0.0;
        for (int j = 0; j < 16; ++j) t += red[j][e];
        out[i] = (float)t;
    }
}

template <int MM>
hipError_t corr_mfma_impl(const Geometry &g, int K, Lists z, const float *r, float *part, int nblk, float *G,
                          hipStream_t s) {
    const int ngroups = (K + CM_FG - 1) / CM_FG;
    SCSC_LAUNCH(k_corr_mfma<MM>, dim3(nblk, ngroups), dim3(TPB), 0, s, g.d_img, g.d_tiles, g.n_tiles, K, z,
                r, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = K * MM * MM;
    SCSC_LAUNCH(k_reduce_f32_partials_f64, dim3((n + 15) / 16), dim3(256), 0, s, part, nblk, n, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis with BF16 operands on the matrix cores (FP32 accumulation and FP32
// residual).  For a 16 x 16 output tile (origin shifted by -c), one GEMM per
// tile forms, for every input row y' of the tile's region and output column x,
//     V[r][y'][x] = sum_k sum_u' d_k[r][2c - u'] z_k[y'][x + u']
//         M = tap row r (padded to 16), N = the 16 output columns,
//         K-dim = (filter, reversed tap column u'), 8 filters x 4 tap columns
//         per 32-wide step;
// the output is the sum over tap rows of V shifted along y:
//     y[ly][lx] = sum_r V[r][ly + 2c - r][lx] = sum_k sum_s d_k[s] z_k[p - s].
// Codes are scattered from the per-pixel lists into a dense BF16 tile of the
// region with the 8 filters of a group innermost, so that one aligned 16-byte
// LDS read gives a lane its 8 operand values; a chunk holds SM_FG groups.
// Operand A comes prepared as dA[r][group][u'][8 filters] (k_synth_prep_a).
// ---------------------------------------------------------------------------
constexpr int SM_CAP = 4096;  // code entries of a region staged in LDS
constexpr int SM_LB = 4;      // list loads in flight per thread while staging

template <int MM>
constexpr int sm_steps() { return (MM + 3) / 4; }  // 4 tap columns per step

template <int MM>
__global__ void k_synth_prep_a(const float *__restrict__ d, int K, __bf16 *__restrict__ dA) {
    constexpr int M = MM * MM, C = MM / 2, U = 4 * sm_steps<MM>();
    const int K8 = (K + 7) / 8;
    const long long n = 16LL * K8 * U * 8;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int f = (int)(i % 8), up = (int)((i / 8) % U);
        const int fg = (int)((i / (8 * U)) % K8), r = (int)(i / (8LL * U * K8));
        const int k = 8 * fg + f, u = 2 * C - up;
        dA[i] = (r < MM && up < MM && k < K) ? (__bf16)d[(long long)k * M + r * MM + u] : (__bf16)0.f;
    }
}

// Exclusive prefix over the block of one int per thread; returns the total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *excl, int *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) {
        before += (w < wave) ? wsum[w] : 0;
        total += wsum[w];
    }
    *excl = before + incl - v;
    return total;
}

template <int MM, int FG>
__global__ __launch_bounds__(TPB, FG == 1 ? 4 : 1) void k_synth_mfma(const ImgInfo *imgs, const TileInfo *tiles, int K, Lists zl,
                                                    const __bf16 *__restrict__ dA, const float *__restrict__ x,
                                                    const unsigned char *__restrict__ W, float *__restrict__ out,
                                                    int mode) {
    constexpr int C = MM / 2, RW = TS + 2 * C, NS = sm_steps<MM>(), U = 4 * NS;
    constexpr int ZC = TS + U - 1;              // columns x + u' that a step reads
    static_assert(ZC >= RW, "code tile narrower than the region");
    constexpr int NPT = (RW * RW + TPB - 1) / TPB;  // region pixels per thread
    constexpr int NCW = (RW + 3) / 4;           // input rows per wave
    constexpr int GT = RW * ZC;                 // 16-byte cells per filter group
    constexpr int ZB = FG * GT * 16;            // bytes of the code tile
    constexpr int LB = ZB + SM_CAP * 6;         // + staged entries (key, value)
    constexpr int VB = 16 * RW * TS;            // floats of the V staging
    static_assert(VB * 4 <= LB, "V staging must fit in the shared buffer");
    __shared__ bf16x8 lds8[LB / 16];
    __shared__ int wsum[TPB / 64];
    bf16x8 *zt8 = lds8;                                   // [group][input row][column][8 filters]
    __bf16 *zt = reinterpret_cast<__bf16 *>(lds8);
    unsigned *skey = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(lds8) + ZB);  // k << 10 | region pixel
    __bf16 *sval = reinterpret_cast<__bf16 *>(skey + SM_CAP);

    const PixelCtx c = pixel_ctx(imgs, tiles, xcd_tile((int)blockIdx.x, (int)gridDim.x));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fcol = lane & 15, kg = lane >> 4;
    const int oy = c.t.ty * TS - C, ox = c.t.tx * TS - C;
    const int K8 = (K + 7) / 8;

    // this thread's region pixels and their lists
    unsigned po[NPT];
    int pn[NPT], ntot = 0;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int i = threadIdx.x + q * TPB;
        const int gy = oy + i / RW, gx = ox + i % RW;
        pn[q] = 0;
        po[q] = 0;
        if (i < RW * RW && gy >= 0 && gy < c.im.H && gx >= 0 && gx < c.im.W) {
            const long long gp = c.im.pix_off + (long long)gy * c.im.W + gx;
            po[q] = zl.off[gp];
            pn[q] = zl.cnt[gp];
        }
        ntot += pn[q];
    }
    int ebeg;
    const int total = block_exclusive_scan(ntot, &ebeg, wsum);
    const bool staged = total <= SM_CAP;  // uniform over the block
    int cur[NPT];  // per-pixel list positions of the unstaged path
#pragma unroll
    for (int q = 0; q < NPT; ++q) cur[q] = 0;
    if (staged) {
        // this thread's entries, flattened over its pixels, SM_LB loads in flight
        for (int j0 = 0; j0 < ntot; j0 += SM_LB) {
            Pair pr[SM_LB];
            unsigned pix[SM_LB];
#pragma unroll
            for (int u = 0; u < SM_LB; ++u) {
                int jj = j0 + u, q = 0;
#pragma unroll
                for (int qq = 0; qq < NPT - 1; ++qq)
                    if (q == qq && jj >= pn[qq]) {
                        jj -= pn[qq];
                        q = qq + 1;
                    }
                unsigned o = po[0];
#pragma unroll
                for (int qq = 1; qq < NPT; ++qq)
                    if (q == qq) o = po[qq];
                pix[u] = threadIdx.x + q * TPB;
                if (j0 + u < ntot) pr[u] = zl.pairs[o + jj];
            }
#pragma unroll
            for (int u = 0; u < SM_LB; ++u)
                if (j0 + u < ntot) {
                    skey[ebeg + j0 + u] = ((unsigned)pr[u].k << 10) | pix[u];
                    sval[ebeg + j0 + u] = (__bf16)pr[u].v;
                }
        }
    }

    const bf16x8 *dA8 = reinterpret_cast<const bf16x8 *>(dA) + (long long)fcol * K8 * U + kg;
    f32x4 acc[NCW];
#pragma unroll
    for (int j = 0; j < NCW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int g0 = 0; g0 < K8; g0 += FG) {
        const int ng = min(FG, K8 - g0);
        // operand A of the whole chunk, issued before the scatter hides its latency
        bf16x8 afr[FG][NS];
#pragma unroll
        for (int gl = 0; gl < FG; ++gl)
#pragma unroll
            for (int st = 0; st < NS; ++st) afr[gl][st] = dA8[(long long)(g0 + min(gl, ng - 1)) * U + 4 * st];
        __syncthreads();  // the previous chunk's operands have been read (and the entries staged)
        for (int i = threadIdx.x; i < FG * GT; i += TPB) zt8[i] = bf16x8{};
        __syncthreads();
        const unsigned k0 = 8 * g0, k1 = min(K, 8 * (g0 + ng));
        if (staged) {
            // all staged entries of the region, strided over the block (balanced), 4 at a time
            for (int e0 = threadIdx.x; e0 < total; e0 += 4 * TPB) {
                unsigned key[4];
                __bf16 val[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * TPB;
                    key[u] = e < total ? skey[e] : 0xffffffffu;
                    val[u] = e < total ? sval[e] : (__bf16)0.f;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const unsigned k = key[u] >> 10;
                    if (k >= k0 && k < k1) {
                        const unsigned kl = k - k0, pix = key[u] & 1023u;
                        const unsigned yr = pix / RW, xr = pix % RW;
                        zt[(((kl >> 3) * RW + yr) * ZC + xr) * 8 + (kl & 7)] = val[u];
                    }
                }
            }
        } else {
            // the lists are sorted by k and the chunks advance in k: one cursor per
            // pixel reads each entry once over the whole loop (plus one look-ahead)
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                const int pix = threadIdx.x + q * TPB;
                const int yr = pix / RW, xr = pix % RW;
                while (cur[q] < pn[q]) {
                    const Pair pr = zl.pairs[po[q] + cur[q]];
                    if ((unsigned)pr.k >= k1) break;
                    const int kl = pr.k - (int)k0;
                    zt[(((kl >> 3) * RW + yr) * ZC + xr) * 8 + (kl & 7)] = (__bf16)pr.v;
                    ++cur[q];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int gl = 0; gl < FG; ++gl) {
            if (gl >= ng) break;
#pragma unroll
            for (int st = 0; st < NS; ++st) {
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw) {
                    const int ct = wave + 4 * cw;  // input row
                    if (ct >= RW) continue;
                    const bf16x8 bfr = zt8[(gl * RW + ct) * ZC + fcol + 4 * st + kg];
                    acc[cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[gl][st], bfr, acc[cw], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();  // the shared buffer becomes the V staging
    float *vb = reinterpret_cast<float *>(lds8);  // [r][input row][column]
#pragma unroll
    for (int cw = 0; cw < NCW; ++cw) {
        const int ct = wave + 4 * cw;
        if (ct >= RW) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) vb[((kg * 4 + i) * RW + ct) * TS + fcol] = acc[cw][i];
    }
    __syncthreads();
    if (!c.valid) return;
    float y = 0.f;
#pragma unroll
    for (int r = 0; r < MM; ++r) y += vb[(r * RW + c.ly + 2 * C - r) * TS + c.lx];
    float ov;
    if (mode == SYNTH_RESIDUAL) {
        ov = x[c.gp] - y;
        if (W && !W[c.gp]) ov = 0.f;
    } else if (mode == SYNTH_WEIGHTED) {
        ov = (W && !W[c.gp]) ? 0.f : y;
    } else {
        ov = y;
    }
    out[c.gp] = ov;
}

template <int MM>
hipError_t synth_mfma_prep_impl(const float *d, int K, __bf16 *dA, hipStream_t s) {
    const long long n = 16LL * ((K + 7) / 8) * 4 * sm_steps<MM>() * 8;
    SCSC_LAUNCH(k_synth_prep_a<MM>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, K, dA);
    return hipGetLastError();
}

template <int MM>
hipError_t synth_mfma_impl(const Geometry &g, int K, Lists z, const __bf16 *dA, const float *x,
                           const unsigned char *W, float *out, int mode, int variant, hipStream_t s) {
    if (variant == 0)
        SCSC_LAUNCH((k_synth_mfma<MM, 2>), dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, z, dA, x, W,
                    out, mode);
    else if (variant == 1)
        SCSC_LAUNCH((k_synth_mfma<MM, 4>), dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, z, dA, x, W,
                    out, mode);
    else
        SCSC_LAUNCH((k_synth_mfma<MM, 1>), dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, z, dA, x, W,
                    out, mode);
    return hipGetLastError();
}

}  // namespace

int corr_mfma_blocks(const Geometry &g, int K) {
    const int ngroups = (K + CM_FG - 1) / CM_FG;
    int nb = 512 / ngroups;
    if (nb < 1) nb = 1;
    return nb < g.n_tiles ? nb : g.n_tiles;
}

size_t synth_mfma_prep_elems(int K) { return (size_t)16 * ((K + 7) / 8) * 12 * 8; }  // up to 12 tap columns

hipError_t launch_synth_mfma_prep(const float *d, int K, int m, __bf16 *dA, hipStream_t s) {
    switch (m) {
        case 3: return synth_mfma_prep_impl<3>(d, K, dA, s);
        case 5: return synth_mfma_prep_impl<5>(d, K, dA, s);
        case 7: return synth_mfma_prep_impl<7>(d, K, dA, s);
        case 9: return synth_mfma_prep_impl<9>(d, K, dA, s);
        case 11: return synth_mfma_prep_impl<11>(d, K, dA, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_synth_mfma(const Geometry &g, int K, int m, Lists z, const __bf16 *dA, const float *x,
                             const unsigned char *W, float *out, int mode, int variant, hipStream_t s) {
    switch (m) {
        case 3: return synth_mfma_impl<3>(g, K, z, dA, x, W, out, mode, variant, s);
        case 5: return synth_mfma_impl<5>(g, K, z, dA, x, W, out, mode, variant, s);
        case 7: return synth_mfma_impl<7>(g, K, z, dA, x, W, out, mode, variant, s);
        case 9: return synth_mfma_impl<9>(g, K, z, dA, x, W, out, mode, variant, s);
        case 11: return synth_mfma_impl<11>(g, K, z, dA, x, W, out, mode, variant, s);
        default: return hipErrorInvalidValue;
    }
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
