// Code-update kernels for gfx950: Bernoulli selection (eq. 2), compact per-pixel
// code lists, the synthesis / masked residual of eq. (3) and one proximal-gradient
// step (adjoint correlation at the selected coordinates + soft-threshold).
//
// Data structures.  For every pixel p of the batch the selected coordinates are a
// bit set over k (mask_words[w][p], w = k / 32).  The codes that are currently
// non-zero are kept as a short list of (k, value) pairs sorted by k, stored at
// [off[p], off[p] + cnt[p]) of a packed pair array; off[] is the exclusive prefix
// of the per-pixel capacity (the number of selected k in a code step, the number
// of non-zeros when lists are built from dense codes).  Since a converged code
// map is very sparse, the synthesis touches only non-zero codes, and the
// proximal step touches only selected coordinates.
#include "scsc_internal.h"

#include <climits>

namespace scsc {

namespace {

// ---------------------------------------------------------------------------
// Selection (eq. 2): one Philox call yields the words of 4 consecutive
// coordinate indices l = (y W + x) K + k.  Thread (pixel, word w) draws the 32
// filters of its mask word (about 8 calls) and adds the word's population to the
// pixel's count (zeroed before the launch), so a pixel's draws run in parallel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_mask_count(const ImgInfo *imgs, int n_img, int K,
                                                    unsigned long long thr, uint2 key, unsigned draw,
                                                    long long n_pix, unsigned *mask_words, unsigned *cnt) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const int kb = (int)blockIdx.y * 32, ke = min(K, kb + 32);
    const unsigned long long base = (unsigned long long)c.p_img * (unsigned long long)K;
    const unsigned long long l0 = base + (unsigned long long)kb, l1 = base + (unsigned long long)ke;
    const bool all = thr > 0xFFFFFFFFull;
    unsigned cur = 0;
    for (unsigned long long g4 = l0 >> 2; (g4 << 2) < l1; ++g4) {
        uint4 w = philox4x32_10(make_uint4((unsigned)g4, (unsigned)(g4 >> 32), (unsigned)c.im.index, draw), key);
        unsigned ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned long long l = (g4 << 2) + j;
            if (l < l0 || l >= l1) continue;
            if (all || (unsigned long long)ws[j] < thr) cur |= 1u << ((int)(l - base) & 31);
        }
    }
    mask_words[(long long)blockIdx.y * n_pix + c.gp] = cur;
    const unsigned n = (unsigned)__popc(cur);
    if (n) atomicAdd(&cnt[c.gp], n);
}

__global__ __launch_bounds__(TPB) void k_expand_mask(const ImgInfo *imgs, const TileInfo *tiles, int K,
                                                     long long n_pix, const unsigned *mask_words,
                                                     unsigned char *mask) {
    PixelCtx c = pixel_ctx(imgs, tiles);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const long long zb = (long long)K * c.im.pix_off + c.p_img;
    unsigned bits = 0;
    for (int k = 0; k < K; ++k) {
        if ((k & 31) == 0) bits = mask_words[(long long)(k >> 5) * n_pix + c.gp];
        mask[zb + (long long)k * HW] = (bits >> (k & 31)) & 1u;
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of per-pixel counts (three passes, 1024 elements per block).
// ---------------------------------------------------------------------------
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = TPB * SCAN_PER_THREAD;

__global__ __launch_bounds__(TPB) void k_scan_local(const unsigned *cnt, unsigned *off, long long n,
                                                    unsigned long long *bsum) {
    __shared__ int scratch[TPB];
    const long long base = (long long)blockIdx.x * SCAN_BLOCK + (long long)threadIdx.x * SCAN_PER_THREAD;
    unsigned v[SCAN_PER_THREAD];
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; ++j) {
        v[j] = (base + j < n) ? cnt[base + j] : 0u;
        s += (int)v[j];
    }
    int total;
    int ex = block_exclusive_scan(s, scratch, &total);
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; ++j) {
        if (base + j < n) off[base + j] = (unsigned)ex;
        ex += (int)v[j];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = (unsigned long long)total;
}

__global__ __launch_bounds__(TPB) void k_scan_blocks(unsigned long long *bsum, long long nb, unsigned *off,
                                                     long long n, unsigned long long *total64) {
    __shared__ unsigned long long sc[TPB];
    unsigned long long carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += TPB) {
        const long long i = b0 + threadIdx.x;
        unsigned long long v = i < nb ? bsum[i] : 0ull;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < TPB; o <<= 1) {
            unsigned long long a = threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
            __syncthreads();
            sc[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sc[threadIdx.x] - v;
        unsigned long long tot = sc[TPB - 1];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total64 = carry;
        off[n] = (unsigned)carry;
    }
}

__global__ __launch_bounds__(TPB) void k_scan_add(unsigned *off, long long n, const unsigned long long *bsum) {
    const long long i = (long long)blockIdx.x * TPB + threadIdx.x;
    if (i < n) off[i] += (unsigned)bsum[i / SCAN_BLOCK];
}

// ---------------------------------------------------------------------------
// Lists from dense codes.
// ---------------------------------------------------------------------------
constexpr int ZB = 8;  // filters (or list entries) per batch of loads in the per-pixel passes over dense z

__global__ __launch_bounds__(TPB) void k_gather_selected(const ImgInfo *imgs, int n_img, int K,
                                                         long long n_pix, const unsigned *mask_words,
                                                         const unsigned *soff, const float *z, Pair *pairs,
                                                         unsigned short *cnt, unsigned long long *nnz_acc) {
    __shared__ int bsum;
    if (threadIdx.x == 0) bsum = 0;
    __syncthreads();
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) {
        __syncthreads();
        if (threadIdx.x == 0 && nnz_acc && bsum) atomicAdd(nnz_acc, (unsigned long long)bsum);
        return;
    }
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = soff[c.gp];
    int nn = 0;
    unsigned bits = 0;
    // ZB filters at a time: their loads are issued together (the lanes of a wave
    // read neighbouring pixels of one filter plane, so every load is coalesced)
    for (int k0 = 0; k0 < K; k0 += ZB) {
        float v[ZB];
#pragma unroll
        for (int u = 0; u < ZB; ++u) v[u] = k0 + u < K ? zp[(long long)(k0 + u) * HW] : 0.f;
#pragma unroll
        for (int u = 0; u < ZB; ++u) {
            const int k = k0 + u;
            if ((k & 31) == 0) bits = k < K ? mask_words[(long long)(k >> 5) * n_pix + c.gp] : 0u;
            if (k < K && ((bits >> (k & 31)) & 1u) && v[u] != 0.f) {
                pairs[base + nn] = Pair{k, v[u]};
                ++nn;
            }
        }
    }
    cnt[c.gp] = (unsigned short)nn;
    if (nn) atomicAdd(&bsum, nn);
    __syncthreads();
    if (threadIdx.x == 0 && nnz_acc && bsum) atomicAdd(nnz_acc, (unsigned long long)bsum);
}

__global__ __launch_bounds__(TPB) void k_count_nonzero(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                       const float *z, unsigned *cnt) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    unsigned nn = 0;
    for (int k0 = 0; k0 < K; k0 += ZB) {
        float v[ZB];
#pragma unroll
        for (int u = 0; u < ZB; ++u) v[u] = k0 + u < K ? zp[(long long)(k0 + u) * HW] : 0.f;
#pragma unroll
        for (int u = 0; u < ZB; ++u) nn += v[u] != 0.f;
    }
    cnt[c.gp] = nn;
}

__global__ __launch_bounds__(TPB) void k_fill_nonzero(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                      const float *z, const unsigned *off, Pair *pairs,
                                                      unsigned short *cnt, XPair *xp, unsigned xmul) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = off[c.gp];
    int nn = 0;
    for (int k0 = 0; k0 < K; k0 += ZB) {
        float v[ZB];
#pragma unroll
        for (int u = 0; u < ZB; ++u) v[u] = k0 + u < K ? zp[(long long)(k0 + u) * HW] : 0.f;
#pragma unroll
        for (int u = 0; u < ZB; ++u) {
            const int k = k0 + u;
            if (v[u] != 0.f) {  // (0 for k >= K)
                pairs[base + nn] = Pair{k, v[u]};
                if (xp) xp[base + nn] = XPair{((unsigned)c.x * xmul + (unsigned)k) * 8u, v[u]};
                ++nn;
            }
        }
    }
    cnt[c.gp] = (unsigned short)nn;
}

// The list lengths of a code step as 32-bit counts (for the exclusive scan).
__global__ __launch_bounds__(TPB) void k_counts_u32(const unsigned short *cnt, long long n, unsigned *out) {
    const long long i = (long long)blockIdx.x * TPB + threadIdx.x;
    if (i < n) out[i] = cnt[i];
}

// Exact-capacity lists (offsets = prefix of the lengths) copied from a code
// step's lists, with the XPair tags of k_fill_nonzero when xp is given.  The
// entries of a pixel keep their order (ascending k), so the result equals what
// k_fill_nonzero builds from the dense codes the lists describe.
__global__ __launch_bounds__(TPB) void k_compact_lists(const ImgInfo *imgs, int n_img, long long n_pix, Lists in,
                                                       const unsigned *off, Pair *pairs, unsigned short *cnt,
                                                       XPair *xp, unsigned xmul) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const unsigned src = in.off[c.gp], dst = off[c.gp];
    const int n = in.cnt[c.gp];
    for (int i0 = 0; i0 < n; i0 += ZB) {
        Pair e[ZB];
#pragma unroll
        for (int u = 0; u < ZB; ++u) e[u] = i0 + u < n ? in.pairs[src + i0 + u] : Pair{0, 0.f};
#pragma unroll
        for (int u = 0; u < ZB; ++u) {
            if (i0 + u >= n) break;
            pairs[dst + i0 + u] = e[u];
            if (xp) xp[dst + i0 + u] = XPair{((unsigned)c.x * xmul + (unsigned)e[u].k) * 8u, e[u].v};
        }
    }
    cnt[c.gp] = (unsigned short)n;
}

__global__ __launch_bounds__(TPB) void k_scatter_dense(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                       Lists zl, float *z) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = zl.off[c.gp];
    const int n = zl.cnt[c.gp];
    // the first ZB entries of the list are loaded together; longer lists continue one by one
    Pair ent[ZB];
#pragma unroll
    for (int u = 0; u < ZB; ++u) ent[u] = u < n ? zl.pairs[base + u] : Pair{INT_MAX, 0.f};
    int i = 0;
    Pair e = ent[0];
    for (int k = 0; k < K; ++k) {
        float v = 0.f;
        if (e.k == k) {
            v = e.v;
            ++i;
            if (i < n) {
                if (i < ZB) {
#pragma unroll
                    for (int u = 1; u < ZB; ++u)
                        if (i == u) e = ent[u];
                } else {
                    e = zl.pairs[base + i];
                }
            } else {
                e = Pair{INT_MAX, 0.f};
            }
        }
        zp[(long long)k * HW] = v;
    }
}

// Held codes (the unselected coordinates keep their values): per pixel, the
// non-zero codes of z whose coordinate is not in the sample (mask words clear).
__global__ __launch_bounds__(TPB) void k_count_held(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                    const unsigned *mask_words, const float *z, unsigned *cnt) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    unsigned nn = 0, bits = 0;
    for (int k = 0; k < K; ++k) {
        if ((k & 31) == 0) bits = mask_words[(long long)(k >> 5) * n_pix + c.gp];
        nn += !((bits >> (k & 31)) & 1u) && zp[(long long)k * HW] != 0.f;
    }
    cnt[c.gp] = nn;
}

__global__ __launch_bounds__(TPB) void k_fill_held(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                   const unsigned *mask_words, const float *z, const unsigned *off,
                                                   Pair *pairs, unsigned short *cnt) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    const float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = off[c.gp];
    unsigned bits = 0;
    int nn = 0;
    for (int k = 0; k < K; ++k) {
        if ((k & 31) == 0) bits = mask_words[(long long)(k >> 5) * n_pix + c.gp];
        if ((bits >> (k & 31)) & 1u) continue;
        const float v = zp[(long long)k * HW];
        if (v != 0.f) {
            pairs[base + nn] = Pair{k, v};
            ++nn;
        }
    }
    cnt[c.gp] = (unsigned short)nn;
}

// z = M^T z~ on the sample only: every selected coordinate takes its list value
// (0 when absent), the unselected coordinates are left as they are.
__global__ __launch_bounds__(TPB) void k_scatter_selected(const ImgInfo *imgs, int n_img, long long n_pix, int K,
                                                          const unsigned *mask_words, Lists zl, float *z) {
    PixelCtx c = flat_ctx(imgs, n_img, n_pix);
    if (!c.valid) return;
    const long long HW = (long long)c.im.H * c.im.W;
    float *zp = z + (long long)K * c.im.pix_off + c.p_img;
    const unsigned base = zl.off[c.gp];
    const int n = zl.cnt[c.gp];
    int i = 0;
    Pair e = n > 0 ? zl.pairs[base] : Pair{INT_MAX, 0.f};
    unsigned bits = 0;
    for (int k = 0; k < K; ++k) {
        if ((k & 31) == 0) bits = mask_words[(long long)(k >> 5) * n_pix + c.gp];
        float v = 0.f;
        if (e.k == k) {
            v = e.v;
            ++i;
            e = i < n ? zl.pairs[base + i] : Pair{INT_MAX, 0.f};
        }
        if ((bits >> (k & 31)) & 1u) zp[(long long)k * HW] = v;
    }
}

__global__ void k_sum_counts(const unsigned short *cnt, long long n, unsigned long long *out) {
    __shared__ unsigned long long red[TPB];
    unsigned long long s = 0;
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < n; i += (long long)gridDim.x * TPB)
        s += cnt[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// ---------------------------------------------------------------------------
// Synthesis from code lists (deterministic gather).
// The tile's output pixels depend on the codes of the tile grown by c pixels.
// Their list headers are staged in LDS, a block scan gives LDS offsets and,
// when the region holds at most SYN_CAP pairs, the pairs themselves are staged.
// Each output pixel then walks its m x m taps in a fixed order.
// ---------------------------------------------------------------------------
// staging capacity (pairs) of a synthesis region: 16-row tiles / 8-row tiles
template <int TY>
constexpr int syn_cap() {
    return TY >= 16 ? 2880 : 2048;
}
constexpr int SYN_DCAP = 12288;  // filters staged in LDS when K m^2 <= 12288 floats (48 KiB)

// A staged code of the synthesis region: filter, region column, value.
struct __align__(8) SynPair {
    int doff;  // k * m^2 - (region column): the code's offset into the filters for tap column 0
    float v;
};

// Synthesis on TT x TY output tiles (TY divides the 16-row geometry tiles) with
// SP threads per output pixel.  The codes of the tile grown by c are staged in
// LDS in region row-major order, so for output p and tap row s_y the codes of
// the 2c + 1 pixels q = p - s form one contiguous run; filters are staged in
// LDS when they fit.  Thread part j of a pixel takes a contiguous range of tap
// rows.  Each tap row's sum is formed the same way for every tile shape and SP,
// and the row sums are added in row order, so the result does not depend on
// the launch variant.  A region whose codes exceed the staging capacity reads
// them from global memory instead, in the same order.
template <int MM, bool DLDS, int TT, int TY, int SP>
__global__ __launch_bounds__(TT *TY *SP) void k_synth(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles, int K,
                                                      Lists zl, const float *__restrict__ d,
                                                      const float *__restrict__ x, const unsigned char *__restrict__ W,
                                                      float *__restrict__ out, int mode) {
    constexpr int C = MM / 2, RW = TT + 2 * C, RH = TY + 2 * C, R = RW * RH, M = MM * MM, NP = TT * TY,
                  NT = NP * SP;
    constexpr int CH = (R + NT - 1) / NT;
    constexpr int RP = (MM + SP - 1) / SP;  // tap rows per part
    constexpr int SUB = TS / TY;            // work items per geometry tile
    constexpr int CAP = syn_cap<TY>();
    __shared__ unsigned lgoff[R];
    __shared__ int lstart[R + 1];
    __shared__ unsigned short lcnt[R];
    __shared__ SynPair lp[CAP];
    __shared__ int scratch[NT];
    __shared__ float rows[SP > 1 ? MM : 1][SP > 1 ? NP : 1];
    __shared__ float dl[DLDS ? SYN_DCAP : 1];

    if (DLDS)
        for (int i = threadIdx.x; i < K * M; i += NT) dl[i] = d[i];
    const float *dd = DLDS ? dl : d;
    const int o = threadIdx.x % NP, part = threadIdx.x / NP;
    const int ly = o / TT, lx = o % TT;
    long long first, step, end;
    xcd_work((long long)n_tiles * SUB, first, step, end);
    for (long long item = first; item < end; item += step) {
        const TileInfo t = tiles[item / SUB];
        const ImgInfo im = imgs[t.img];
        const int y0 = t.ty * TS + (int)(item % SUB) * TY, x0 = t.tx * TT;
        if (y0 >= im.H) continue;  // work item below the image (uniform over the workgroup)
        __syncthreads();           // LDS of the previous item is no longer read
        const int y = y0 + ly, xx = x0 + lx;
        const bool valid = y < im.H && xx < im.W;
        const int oy = y0 - C, ox = x0 - C;
        int mysum = 0;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int i = threadIdx.x * CH + j;
            if (i < R) {
                const int gy = oy + i / RW, gx = ox + i % RW;
                int n = 0;
                unsigned off = 0;
                if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) {
                    const long long gp = im.pix_off + (long long)gy * im.W + gx;
                    n = zl.cnt[gp];
                    off = zl.off[gp];
                }
                lcnt[i] = (unsigned short)n;
                lgoff[i] = off;
                mysum += n;
            }
        }
        int total;
        int ex = block_exclusive_scan_n<NT>(mysum, scratch, &total);
        const bool staged = total <= CAP;
        // staging: the first SB codes of every region pixel of this thread are loaded
        // together (independent loads in flight), longer lists finish in a loop
        constexpr int SB = 6;
        Pair pre[CH][SB];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int i = threadIdx.x * CH + j;
            const int n = i < R && staged ? (int)lcnt[i] : 0;
            const Pair *src = zl.pairs + (i < R ? lgoff[i] : 0u);
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q < n) pre[j][q] = src[q];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int i = threadIdx.x * CH + j;
            if (i < R) {
                lstart[i] = ex;
                const int n = lcnt[i];
                if (staged) {
                    const int col = i % RW;
#pragma unroll
                    for (int q = 0; q < SB; ++q)
                        if (q < n) lp[ex + q] = SynPair{pre[j][q].k * M - col, pre[j][q].v};
                    for (int q = SB; q < n; ++q) {
                        const Pair e = zl.pairs[lgoff[i] + q];
                        lp[ex + q] = SynPair{e.k * M - col, e.v};
                    }
                }
                ex += n;
            }
        }
        if (threadIdx.x == 0) lstart[R] = total;
        __syncthreads();
        float acc = 0.f;
        if (valid) {
            const int r0 = part * RP, r1 = r0 + RP < MM ? r0 + RP : MM;
            for (int r = r0; r < r1; ++r) {
                const int sy = r - C;
                float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
                const int rb = (ly + C - sy) * RW + lx;
                if (staged) {
                    const int j0 = lstart[rb], j1 = lstart[rb + 2 * C + 1];
                    const float *drow = dd + r * MM + 2 * C + lx;  // tap column = 2c - (col - lx)
                    int j = j0;
                    // eight elements per step, element j - j0 into accumulator (j - j0) mod 4
                    for (; j + 7 < j1; j += 8) {
                        const SynPair e0 = lp[j], e1 = lp[j + 1], e2 = lp[j + 2], e3 = lp[j + 3];
                        const SynPair e4 = lp[j + 4], e5 = lp[j + 5], e6 = lp[j + 6], e7 = lp[j + 7];
                        const float f0 = drow[e0.doff], f1 = drow[e1.doff], f2 = drow[e2.doff], f3 = drow[e3.doff];
                        const float f4 = drow[e4.doff], f5 = drow[e5.doff], f6 = drow[e6.doff], f7 = drow[e7.doff];
                        a0 = fmaf(f0, e0.v, a0);
                        a1 = fmaf(f1, e1.v, a1);
                        a2 = fmaf(f2, e2.v, a2);
                        a3 = fmaf(f3, e3.v, a3);
                        a0 = fmaf(f4, e4.v, a0);
                        a1 = fmaf(f5, e5.v, a1);
                        a2 = fmaf(f6, e6.v, a2);
                        a3 = fmaf(f7, e7.v, a3);
                    }
                    if (j + 3 < j1) {
                        const SynPair e0 = lp[j], e1 = lp[j + 1], e2 = lp[j + 2], e3 = lp[j + 3];
                        a0 = fmaf(drow[e0.doff], e0.v, a0);
                        a1 = fmaf(drow[e1.doff], e1.v, a1);
                        a2 = fmaf(drow[e2.doff], e2.v, a2);
                        a3 = fmaf(drow[e3.doff], e3.v, a3);
                        j += 4;
                    }
                    // tail: element j - j0 goes to accumulator (j - j0) mod 4 as in the loop
                    if (j < j1) a0 = fmaf(drow[lp[j].doff], lp[j].v, a0);
                    if (j + 1 < j1) a1 = fmaf(drow[lp[j + 1].doff], lp[j + 1].v, a1);
                    if (j + 2 < j1) a2 = fmaf(drow[lp[j + 2].doff], lp[j + 2].v, a2);
                } else {
                    // same elements in the same order; b0 always takes the next element and the
                    // four accumulators rotate, so element u lands in accumulator u mod 4
                    float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
                    int u = 0;
                    for (int w = 0; w < MM; ++w) {
                        const int n = lcnt[rb + w];
                        const Pair *src = zl.pairs + lgoff[rb + w];
                        const float *dt = dd + r * MM + (MM - 1 - w);
                        for (int q = 0; q < n; ++q, ++u) {
                            const Pair e = src[q];
                            const float nb = fmaf(dt[e.k * M], e.v, b0);
                            b0 = b1;
                            b1 = b2;
                            b2 = b3;
                            b3 = nb;
                        }
                    }
                    // b_i now holds accumulator (u + i) mod 4
                    switch (u & 3) {
                        case 0: a0 = b0; a1 = b1; a2 = b2; a3 = b3; break;
                        case 1: a1 = b0; a2 = b1; a3 = b2; a0 = b3; break;
                        case 2: a2 = b0; a3 = b1; a0 = b2; a1 = b3; break;
                        default: a3 = b0; a0 = b1; a1 = b2; a2 = b3; break;
                    }
                }
                const float rs = (a0 + a1) + (a2 + a3);
                if (SP > 1) rows[r][o] = rs;
                else acc += rs;
            }
        }
        if (SP > 1) {
            __syncthreads();
            if (part == 0 && valid)
                for (int r = 0; r < MM; ++r) acc += rows[r][o];
        }
        if (part == 0 && valid) {
            const long long gp = im.pix_off + (long long)y * im.W + xx;
            float ov;
            if (mode == SYNTH_RESIDUAL) {
                ov = x[gp] - acc;
                if (W && !W[gp]) ov = 0.f;
            } else if (mode == SYNTH_WEIGHTED) {
                ov = (W && !W[gp]) ? 0.f : acc;
            } else {
                ov = acc;
            }
            out[gp] = ov;
        }
    }
}

constexpr int ADJ_CAP = 2048;

// Copy a short code list into LDS with its first eight loads issued together.
__device__ __forceinline__ void stage_pairs(const Pair *__restrict__ src, int n, Pair *dst) {
    Pair t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < n) t[q] = src[q];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < n) dst[q] = t[q];
    for (int q = 8; q < n; ++q) dst[q] = src[q];
}

// Dot product of an LDS filter row (float4-aligned, zero padded) with the
// register window.
template <int M4>
__device__ __forceinline__ float dot_window(const float4 *dr, const float (&win)[M4]) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int j = 0; j < M4 / 4; ++j) {
        const float4 q = dr[j];
        a0 = fmaf(q.x, win[4 * j + 0], a0);
        a1 = fmaf(q.y, win[4 * j + 1], a1);
        a2 = fmaf(q.z, win[4 * j + 2], a2);
        a3 = fmaf(q.w, win[4 * j + 3], a3);
    }
    return (a0 + a1) + (a2 + a3);
}

template <int MM>
__global__ __launch_bounds__(TPB) void k_adjoint_shrink(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles,
                                                        int K, long long n_pix, const unsigned *__restrict__ mask_words,
                                                        const unsigned *__restrict__ soff,
                                                        const Pair *__restrict__ oldp,
                                                        const unsigned short *__restrict__ oldc,
                                                        Pair *__restrict__ newp, unsigned short *__restrict__ newc,
                                                        const float *__restrict__ r, const float *__restrict__ d,
                                                        const float *__restrict__ ethr, int KC,
                                                        unsigned long long *__restrict__ nnz_acc) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM, M4 = (M + 3) / 4 * 4;
    __shared__ float rr[RW * RW];
    __shared__ Pair op[ADJ_CAP];
    __shared__ int scratch[TPB];
    __shared__ int bsum;
    extern __shared__ float4 dl4[];
    float *dl = reinterpret_cast<float *>(dl4);
    const float eta = ethr[0], thr = ethr[1];
    const bool one_chunk = K <= KC;
    if (threadIdx.x == 0) bsum = 0;
    if (one_chunk)
        for (int i = threadIdx.x; i < K * M4; i += TPB) {
            const int kk = i / M4, j = i % M4;
            dl[i] = j < M ? d[(long long)kk * M + j] : 0.f;
        }
    long long first, step, end;
    xcd_work(n_tiles, first, step, end);
    for (long long tile = first; tile < end; tile += step) {
        PixelCtx c = pixel_ctx(imgs, tiles, (int)tile);
        __syncthreads();  // LDS of the previous tile is no longer read
        const int oy = c.t.ty * TS - C, ox = c.t.tx * TS - C;
        for (int i = threadIdx.x; i < RW * RW; i += TPB) {
            const int gy = oy + i / RW, gx = ox + i % RW;
            float v = 0.f;
            if (gy >= 0 && gy < c.im.H && gx >= 0 && gx < c.im.W) v = r[c.im.pix_off + (long long)gy * c.im.W + gx];
            rr[i] = v;
        }
        const unsigned base = c.valid ? soff[c.gp] : 0u;
        const int ocnt = c.valid ? (int)oldc[c.gp] : 0;
        int total;
        const int ex = block_exclusive_scan(ocnt, scratch, &total);
        const bool staged = total <= ADJ_CAP;
        if (staged) stage_pairs(oldp + base, ocnt, op + ex);
        __syncthreads();
        float win[M4];
#pragma unroll
        for (int j = 0; j < M4; ++j) {
            if (j < M) {
                const int sy = j / MM - C, sx = j % MM - C;
                win[j] = rr[(c.ly + C + sy) * RW + (c.lx + C + sx)];
            } else {
                win[j] = 0.f;
            }
        }
        int oi = 0;
        Pair oe = ocnt > 0 ? (staged ? op[ex] : oldp[base]) : Pair{INT_MAX, 0.f};
        int nn = 0;
        for (int k0 = 0; k0 < K; k0 += KC) {
            const int k1 = min(K, k0 + KC);
            if (!one_chunk) {
                __syncthreads();
                for (int i = threadIdx.x; i < (k1 - k0) * M4; i += TPB) {
                    const int kk = i / M4, j = i % M4;
                    dl[i] = j < M ? d[(long long)(k0 + kk) * M + j] : 0.f;
                }
                __syncthreads();
            }
            if (!c.valid) continue;
            for (int w = k0 >> 5; w <= (k1 - 1) >> 5; ++w) {
                unsigned bits = mask_words[(long long)w * n_pix + c.gp];
                const int lo = k0 - 32 * w, hi = k1 - 32 * w;
                if (lo > 0) bits &= ~0u << lo;
                if (hi < 32) bits &= (1u << hi) - 1u;
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    const int k = 32 * w + b;
                    while (oe.k < k) {
                        ++oi;
                        oe = oi < ocnt ? (staged ? op[ex + oi] : oldp[base + oi]) : Pair{INT_MAX, 0.f};
                    }
                    float zold = 0.f;
                    if (oe.k == k) {
                        zold = oe.v;
                        ++oi;
                        oe = oi < ocnt ? (staged ? op[ex + oi] : oldp[base + oi]) : Pair{INT_MAX, 0.f};
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    const float g = dot_window<M4>(dl4 + (k - k0) * (M4 / 4), win);
                    const float v = soft_threshold(fmaf(eta, g, zold), thr);
                    if (v != 0.f) {
                        newp[base + nn] = Pair{k, v};
                        ++nn;
                    }
                }
            }
        }
        if (c.valid) newc[c.gp] = (unsigned short)nn;
        if (nn) atomicAdd(&bsum, nn);
    }
    __syncthreads();
    if (threadIdx.x == 0 && nnz_acc && bsum) atomicAdd(nnz_acc, (unsigned long long)bsum);
}

// Dense adjoint D^T r at every coordinate.  Thread <-> pixel with its residual
// window in registers; all lanes walk the same k, so filter reads from LDS are
// broadcasts and the stores of one k are coalesced.
// ---------------------------------------------------------------------------
// BF16 variant of the proximal-gradient iteration: the adjoint correlation of
// the whole 16 x 16 tile is an implicit-im2col GEMM on the matrix cores,
//     G[k][q] = sum_t d_k[t] r[q + t]   (M = filters, N = the tile's pixels,
//                                        K-dim = the m^2 taps padded to 32s),
// with both operands rounded to BF16 (round to nearest even) and FP32
// accumulation (v_mfma_f32_16x16x32_bf16).  Wave w owns pixel rows 4w..4w+3 (four
// 16-pixel column tiles) and keeps their im2col fragments in registers; filters
// are taken 32 at a time, their G written to LDS, and the same selected-set
// epilogue as the FP32 kernel (u = z + eta g, shrink, new lists) reads it there.
// The filters come prepared as dA[k][32 ceil(m^2 / 32)] (BF16, taps zero padded,
// rows padded to a multiple of 32 with zeros), so every lane loads its operand
// fragments directly.  Two variants with the same arithmetic: PF loads the next
// chunk's operand fragments during the current chunk (204 registers, two
// workgroups per CU); without PF they load at the chunk's start (168 registers,
// three workgroups per CU), which runs better beside other kernels.
// Fragment layout of the 16x16x32 instruction (lane l, element i):
//   A: row l % 16, k 8 (l / 16) + i;  B: k 8 (l / 16) + i, column l % 16;
//   D: row 4 (l / 16) + i, column l % 16.
// ---------------------------------------------------------------------------
constexpr int MF_KB = 32;  // filters per chunk
constexpr int MF_MW = 4;   // selection words kept in registers (K <= 128)

template <int MM>
__global__ void k_adj_prep_a(const float *__restrict__ d, int K, int Kp, __bf16 *__restrict__ dA) {
    constexpr int M = MM * MM, MP = 32 * ((M + 31) / 32);
    const long long n = (long long)Kp * MP;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(i / MP), t = (int)(i % MP);
        dA[i] = (k < K && t < M) ? (__bf16)d[(long long)k * M + t] : (__bf16)0.f;
    }
}

template <int MM, bool PF>
__global__ __launch_bounds__(TPB, PF ? 1 : 3) void k_adjoint_shrink_mfma(const ImgInfo *imgs, const TileInfo *tiles, int K,
                                                             long long n_pix, const unsigned *__restrict__ mask_words,
                                                             const unsigned *__restrict__ soff,
                                                             const Pair *__restrict__ oldp,
                                                             const unsigned short *__restrict__ oldc,
                                                             Pair *__restrict__ newp,
                                                             unsigned short *__restrict__ newc,
                                                             const float *__restrict__ r,
                                                             const __bf16 *__restrict__ dA,
                                                             const float *__restrict__ ethr,
                                                             unsigned long long *__restrict__ nnz_acc) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM, NKS = (M + 31) / 32, MP = 32 * NKS;
    __shared__ __bf16 rb[RW * RW];
    __shared__ float gc[MF_KB][TPB];       // G of the chunk, [filter][tile pixel]
    __shared__ Pair op[ADJ_CAP];
    __shared__ int scratch[TPB];
    __shared__ int bsum;

    const float eta = ethr[0], thr = ethr[1];
    PixelCtx c = pixel_ctx(imgs, tiles, xcd_tile((int)blockIdx.x, (int)gridDim.x));
    const int oy = c.t.ty * TS - C, ox = c.t.tx * TS - C;
    for (int i = threadIdx.x; i < RW * RW; i += TPB) {
        const int gy = oy + i / RW, gx = ox + i % RW;
        float v = 0.f;
        if (gy >= 0 && gy < c.im.H && gx >= 0 && gx < c.im.W) v = r[c.im.pix_off + (long long)gy * c.im.W + gx];
        rb[i] = (__bf16)v;
    }
    const unsigned base = c.valid ? soff[c.gp] : 0u;
    const int ocnt = c.valid ? (int)oldc[c.gp] : 0;
    int total;
    const int ex = block_exclusive_scan(ocnt, scratch, &total);
    const bool staged = total <= ADJ_CAP;
    if (staged) stage_pairs(oldp + base, ocnt, op + ex);
    __syncthreads();

    // im2col fragments of this wave's four column tiles (pixel rows 4w..4w+3)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fcol = lane & 15, fk = 8 * (lane >> 4);
    bf16x8 bfr[4][NKS];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int py = wave * 4 + ct;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int t = ks * 32 + fk + i;
                bfr[ct][ks][i] = t < M ? rb[(py + t / MM) * RW + fcol + t % MM] : (__bf16)0.f;
            }
        }
    }

    int oi = 0;
    Pair oe = ocnt > 0 ? (staged ? op[ex] : oldp[base]) : Pair{INT_MAX, 0.f};
    int nn = 0;
    // the pixel's first MF_MW selection words, loaded once
    unsigned mwr[MF_MW];
#pragma unroll
    for (int w = 0; w < MF_MW; ++w) mwr[w] = (c.valid && 32 * w < K) ? mask_words[(long long)w * n_pix + c.gp] : 0u;
    // operand A of a chunk: rows k0 + 16 rt + fcol, K-dim 32 ks + 8 (lane / 16)
    const bf16x8 *dA8 = reinterpret_cast<const bf16x8 *>(dA) + (long long)fcol * (MP / 8) + (lane >> 4);
    bf16x8 afr[2][NKS], afn[2][NKS];
    if constexpr (PF) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) afn[rt][ks] = dA8[(long long)(rt * 16) * (MP / 8) + ks * 4];
    }
    for (int k0 = 0; k0 < K; k0 += MF_KB) {
        const int nk = min(MF_KB, K - k0);
        if constexpr (PF) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) afr[rt][ks] = afn[rt][ks];
            if (k0 + MF_KB < K)  // the next chunk's operands load during this chunk
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ks = 0; ks < NKS; ++ks)
                        afn[rt][ks] = dA8[(long long)(k0 + MF_KB + rt * 16) * (MP / 8) + ks * 4];
        } else {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) afr[rt][ks] = dA8[(long long)(k0 + rt * 16) * (MP / 8) + ks * 4];
        }
        // gc is wave-private: wave w writes G for the tile pixels 64w .. 64w + 63 (its
        // four pixel rows) and only its own threads read them in the epilogue.  The LDS
        // performs one wave's accesses in issue order, so a wavefront-scope fence (which
        // keeps the compiler from moving them) replaces the workgroup barriers here, and
        // the waves of a tile no longer wait for each other between chunks
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            if (rt * 16 < nk) {  // (a guard, not a break: the loop stays unrolled)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < NKS; ++ks)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[rt][ks], bfr[ct][ks], acc, 0, 0, 0);
                    const int px = (wave * 4 + ct) * TS + fcol;
#pragma unroll
                    for (int i = 0; i < 4; ++i) gc[rt * 16 + (lane >> 4) * 4 + i][px] = acc[i];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (!c.valid) continue;
        const int k1 = k0 + nk;
        for (int w = k0 >> 5; w <= (k1 - 1) >> 5; ++w) {
            unsigned bits = 0u;
#pragma unroll
            for (int q = 0; q < MF_MW; ++q)
                if (q == w) bits = mwr[q];
            if (w >= MF_MW) bits = mask_words[(long long)w * n_pix + c.gp];
            const int lo = k0 - 32 * w, hi = k1 - 32 * w;
            if (lo > 0) bits &= ~0u << lo;
            if (hi < 32) bits &= (1u << hi) - 1u;
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const int k = 32 * w + b;
                while (oe.k < k) {
                    ++oi;
                    oe = oi < ocnt ? (staged ? op[ex + oi] : oldp[base + oi]) : Pair{INT_MAX, 0.f};
                }
                float zold = 0.f;
                if (oe.k == k) {
                    zold = oe.v;
                    ++oi;
                    oe = oi < ocnt ? (staged ? op[ex + oi] : oldp[base + oi]) : Pair{INT_MAX, 0.f};
                }
                const float v = soft_threshold(fmaf(eta, gc[k - k0][threadIdx.x], zold), thr);
                if (v != 0.f) {
                    newp[base + nn] = Pair{k, v};
                    ++nn;
                }
            }
        }
    }
    if (c.valid) newc[c.gp] = (unsigned short)nn;
    if (threadIdx.x == 0) bsum = 0;
    __syncthreads();
    if (nn) atomicAdd(&bsum, nn);
    __syncthreads();
    if (threadIdx.x == 0 && nnz_acc && bsum) atomicAdd(nnz_acc, (unsigned long long)bsum);
}

template <int MM>
__global__ __launch_bounds__(TPB) void k_adjoint_dense(const ImgInfo *imgs, const TileInfo *tiles, int K,
                                                       const float *__restrict__ r, const float *__restrict__ d,
                                                       float *__restrict__ out, int KC) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM, M4 = (M + 3) / 4 * 4;
    __shared__ float rr[RW * RW];
    extern __shared__ float4 dl4[];
    float *dl = reinterpret_cast<float *>(dl4);
    PixelCtx c = pixel_ctx(imgs, tiles);
    const int oy = c.t.ty * TS - C, ox = c.t.tx * TS - C;
    for (int i = threadIdx.x; i < RW * RW; i += TPB) {
        const int gy = oy + i / RW, gx = ox + i % RW;
        float v = 0.f;
        if (gy >= 0 && gy < c.im.H && gx >= 0 && gx < c.im.W) v = r[c.im.pix_off + (long long)gy * c.im.W + gx];
        rr[i] = v;
    }
    __syncthreads();
    float win[M4];
#pragma unroll
    for (int j = 0; j < M4; ++j) {
        if (j < M) {
            const int sy = j / MM - C, sx = j % MM - C;
            win[j] = rr[(c.ly + C + sy) * RW + (c.lx + C + sx)];
        } else {
            win[j] = 0.f;
        }
    }
    const long long HW = (long long)c.im.H * c.im.W;
    float *op = out + (long long)K * c.im.pix_off + c.p_img;
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int k1 = min(K, k0 + KC);
        __syncthreads();
        for (int i = threadIdx.x; i < (k1 - k0) * M4; i += TPB) {
            const int kk = i / M4, j = i % M4;
            dl[i] = j < M ? d[(long long)(k0 + kk) * M + j] : 0.f;
        }
        __syncthreads();
        if (!c.valid) continue;
        for (int k = k0; k < k1; ++k) op[(long long)k * HW] = dot_window<M4>(dl4 + (k - k0) * (M4 / 4), win);
    }
}

// Dense adjoint g = D^T r at every coordinate with BF16 operands on the matrix
// cores: the same implicit-im2col GEMM per 16 x 16 tile as the selected-set
// kernel (M = filters, N = the tile's pixels, K-dim = the m^2 taps padded to 32s,
// FP32 accumulation), with the accumulators stored straight to out[k][H][W]:
// lane l holds filters 4 (l / 16) + i of pixel column l % 16, so 16 lanes write
// 64 contiguous bytes of one filter plane.  Filters come from k_adj_prep_a.
template <int MM>
__global__ __launch_bounds__(TPB) void k_adjoint_dense_mfma(const ImgInfo *imgs, const TileInfo *tiles, int n_tiles,
                                                            int K, const float *__restrict__ r,
                                                            const __bf16 *__restrict__ dA, float *__restrict__ out) {
    constexpr int C = MM / 2, RW = TS + 2 * C, M = MM * MM, NKS = (M + 31) / 32, MP = 32 * NKS;
    __shared__ __bf16 rb[RW * RW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fcol = lane & 15, fk = 8 * (lane >> 4);
    const bf16x8 *dA8 = reinterpret_cast<const bf16x8 *>(dA) + (long long)fcol * (MP / 8) + (lane >> 4);
    long long first, step, end;
    xcd_work(n_tiles, first, step, end);
    for (long long tile = first; tile < end; tile += step) {
        const TileInfo t = tiles[tile];
        const ImgInfo im = imgs[t.img];
        const int oy = t.ty * TS - C, ox = t.tx * TS - C;
        __syncthreads();  // the previous tile's fragments have been read
        for (int i = threadIdx.x; i < RW * RW; i += TPB) {
            const int gy = oy + i / RW, gx = ox + i % RW;
            float v = 0.f;
            if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) v = r[im.pix_off + (long long)gy * im.W + gx];
            rb[i] = (__bf16)v;
        }
        __syncthreads();
        bf16x8 bfr[4][NKS];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int py = wave * 4 + ct;
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int tp = ks * 32 + fk + i;
                    bfr[ct][ks][i] = tp < M ? rb[(py + tp / MM) * RW + fcol + tp % MM] : (__bf16)0.f;
                }
            }
        }
        const long long HW = (long long)im.H * im.W;
        const int gx = t.tx * TS + fcol;
        float *ob = out + (long long)K * im.pix_off;
        for (int k0 = 0; k0 < K; k0 += 16) {
            bf16x8 afr[NKS];
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) afr[ks] = dA8[(long long)k0 * (MP / 8) + ks * 4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[ks], bfr[ct][ks], acc, 0, 0, 0);
                const int gy = t.ty * TS + wave * 4 + ct;
                if (gy < im.H && gx < im.W) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = k0 + (lane >> 4) * 4 + i;
                        if (k < K) ob[(long long)k * HW + (long long)gy * im.W + gx] = acc[i];
                    }
                }
            }
        }
    }
}

// Filters per LDS chunk: at most 56 KiB of staged filters, a multiple of 4.
template <int MM>
int filter_chunk() {
    constexpr int M = MM * MM, M4 = (M + 3) / 4 * 4;
    int kc = (52 * 1024) / (M4 * 4);
    kc = kc / 4 * 4;
    return kc > MAX_K ? MAX_K : kc;
}

}  // namespace

#define SCSC_DISPATCH_M(m, FN, ...)         \
    switch (m) {                            \
        case 3: return FN<3>(__VA_ARGS__);  \
        case 5: return FN<5>(__VA_ARGS__);  \
        case 7: return FN<7>(__VA_ARGS__);  \
        case 9: return FN<9>(__VA_ARGS__);  \
        case 11: return FN<11>(__VA_ARGS__); \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_mask_count(const Geometry &g, int K, unsigned long long thr, unsigned long long seed,
                             unsigned draw, unsigned *mask_words, unsigned *cnt, hipStream_t s) {
    uint2 key = make_uint2((unsigned)seed, (unsigned)(seed >> 32));
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(unsigned) * (size_t)g.n_pix, s);
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_mask_count, dim3(flat_grid(g.n_pix), (unsigned)((K + 31) / 32)), dim3(TPB), 0, s, g.d_img,
                g.n_img, K, thr, key, draw, g.n_pix, mask_words, cnt);
    return hipGetLastError();
}

hipError_t launch_expand_mask(const Geometry &g, int K, const unsigned *mask_words, unsigned char *mask,
                              hipStream_t s) {
    SCSC_LAUNCH(k_expand_mask, dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K, g.n_pix,
                mask_words, mask);
    return hipGetLastError();
}

long long scan_tmp_elems(long long n) { return (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1; }

hipError_t launch_scan(const unsigned *cnt, unsigned *off, long long n, unsigned long long *tmp,
                       unsigned long long *total64, hipStream_t s) {
    const long long nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb > 0) SCSC_LAUNCH(k_scan_local, dim3((unsigned)nb), dim3(TPB), 0, s, cnt, off, n, tmp);
    SCSC_LAUNCH(k_scan_blocks, dim3(1), dim3(TPB), 0, s, tmp, nb, off, n, total64);
    if (n > 0) SCSC_LAUNCH(k_scan_add, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, off, n, tmp);
    return hipGetLastError();
}

hipError_t launch_gather_selected(const Geometry &g, int K, const unsigned *mask_words, const unsigned *soff,
                                  const float *z, Pair *pairs, unsigned short *cnt, unsigned long long *nnz_acc,
                                  hipStream_t s) {
    SCSC_LAUNCH(k_gather_selected, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, K, g.n_pix,
                mask_words, soff, z, pairs, cnt, nnz_acc);
    return hipGetLastError();
}

hipError_t launch_count_nonzero(const Geometry &g, int K, const float *z, unsigned *cnt, hipStream_t s) {
    SCSC_LAUNCH(k_count_nonzero, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K, z,
                cnt);
    return hipGetLastError();
}

hipError_t launch_fill_nonzero(const Geometry &g, int K, const float *z, const unsigned *off, Pair *pairs,
                               unsigned short *cnt, XPair *xp, unsigned xmul, hipStream_t s) {
    SCSC_LAUNCH(k_fill_nonzero, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K, z,
                off, pairs, cnt, xp, xmul);
    return hipGetLastError();
}

hipError_t launch_counts_u32(const unsigned short *cnt, long long n, unsigned *out, hipStream_t s) {
    SCSC_LAUNCH(k_counts_u32, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, cnt, n, out);
    return hipGetLastError();
}

hipError_t launch_compact_lists(const Geometry &g, Lists in, const unsigned *off, Pair *pairs, unsigned short *cnt,
                                XPair *xp, unsigned xmul, hipStream_t s) {
    SCSC_LAUNCH(k_compact_lists, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, in, off,
                pairs, cnt, xp, xmul);
    return hipGetLastError();
}

hipError_t launch_scatter_dense(const Geometry &g, int K, Lists z, float *zout, hipStream_t s) {
    SCSC_LAUNCH(k_scatter_dense, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K, z,
                zout);
    return hipGetLastError();
}

hipError_t launch_count_held(const Geometry &g, int K, const unsigned *mask_words, const float *z, unsigned *cnt,
                             hipStream_t s) {
    SCSC_LAUNCH(k_count_held, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K,
                mask_words, z, cnt);
    return hipGetLastError();
}

hipError_t launch_fill_held(const Geometry &g, int K, const unsigned *mask_words, const float *z, const unsigned *off,
                            Pair *pairs, unsigned short *cnt, hipStream_t s) {
    SCSC_LAUNCH(k_fill_held, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K,
                mask_words, z, off, pairs, cnt);
    return hipGetLastError();
}

hipError_t launch_scatter_selected(const Geometry &g, int K, const unsigned *mask_words, Lists zl, float *z,
                                   hipStream_t s) {
    SCSC_LAUNCH(k_scatter_selected, dim3(flat_grid(g.n_pix)), dim3(TPB), 0, s, g.d_img, g.n_img, g.n_pix, K,
                mask_words, zl, z);
    return hipGetLastError();
}

hipError_t launch_sum_counts(const unsigned short *cnt, long long n, unsigned long long *out, hipStream_t s) {
    long long nb = (n + TPB - 1) / TPB;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    SCSC_LAUNCH(k_sum_counts, dim3((unsigned)nb), dim3(TPB), 0, s, cnt, n, out);
    return hipGetLastError();
}

namespace {
template <int MM, bool DLDS, int TY, int SP>
hipError_t synth_launch(const Geometry &g, int K, Lists z, const float *d, const float *x, const unsigned char *W,
                        float *out, SynthMode mode, hipStream_t s) {
    const void *kfn = reinterpret_cast<const void *>(&k_synth<MM, DLDS, TS, TY, SP>);
    const int block = TS * TY * SP;
    const int grid = persistent_grid(kfn, block, 0, (long long)g.n_tiles * (TS / TY));
    SCSC_LAUNCH((k_synth<MM, DLDS, TS, TY, SP>), dim3(grid), dim3(block), 0, s, g.d_img, g.d_tiles, g.n_tiles,
                K, z, d, x, W, out, (int)mode);
    return hipGetLastError();
}

template <int MM, int TY, int SP>
hipError_t synth_sp(const Geometry &g, int K, Lists z, const float *d, const float *x, const unsigned char *W,
                    float *out, SynthMode mode, hipStream_t s) {
    if (K * MM * MM <= SYN_DCAP) return synth_launch<MM, true, TY, SP>(g, K, z, d, x, W, out, mode, s);
    return synth_launch<MM, false, TY, SP>(g, K, z, d, x, W, out, mode, s);
}

template <int MM>
hipError_t synth_impl(const Geometry &g, int K, Lists z, const float *d, const float *x, const unsigned char *W,
                      float *out, SynthMode mode, int variant, hipStream_t s) {
    switch (variant) {
        case 1: return synth_sp<MM, 16, 4>(g, K, z, d, x, W, out, mode, s);
        case 2: return synth_sp<MM, 8, 2>(g, K, z, d, x, W, out, mode, s);
        case 3: return synth_sp<MM, 8, 4>(g, K, z, d, x, W, out, mode, s);
        default: return synth_sp<MM, 16, 1>(g, K, z, d, x, W, out, mode, s);
    }
}

template <int MM>
hipError_t adjoint_shrink_impl(const Geometry &g, int K, const unsigned *mw, const unsigned *soff,
                               const Pair *oldp, const unsigned short *oldc, Pair *newp, unsigned short *newc,
                               const float *r, const float *d, const float *ethr, unsigned long long *nnz_acc,
                               hipStream_t s) {
    constexpr int M = MM * MM, M4 = (M + 3) / 4 * 4;
    const int KC = filter_chunk<MM>();
    const int kc = K < KC ? K : KC;
    const size_t shm = (size_t)kc * M4 * sizeof(float);
    const int grid = persistent_grid(reinterpret_cast<const void *>(&k_adjoint_shrink<MM>), TPB, shm, g.n_tiles);
    SCSC_LAUNCH(k_adjoint_shrink<MM>, dim3(grid), dim3(TPB), shm, s, g.d_img, g.d_tiles, g.n_tiles, K,
                g.n_pix, mw, soff, oldp, oldc, newp, newc, r, d, ethr, KC, nnz_acc);
    return hipGetLastError();
}

template <int MM>
hipError_t adjoint_shrink_mfma_impl(const Geometry &g, int K, const unsigned *mw, const unsigned *soff,
                                    const Pair *oldp, const unsigned short *oldc, Pair *newp, unsigned short *newc,
                                    const float *r, const __bf16 *dA, const float *ethr,
                                    unsigned long long *nnz_acc, int variant, hipStream_t s) {
    if (variant == 0)
        SCSC_LAUNCH((k_adjoint_shrink_mfma<MM, true>), dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles, K,
                    g.n_pix, mw, soff, oldp, oldc, newp, newc, r, dA, ethr, nnz_acc);
    else
        SCSC_LAUNCH((k_adjoint_shrink_mfma<MM, false>), dim3(g.n_tiles), dim3(TPB), 0, s, g.d_img, g.d_tiles,
                    K, g.n_pix, mw, soff, oldp, oldc, newp, newc, r, dA, ethr, nnz_acc);
    return hipGetLastError();
}

template <int MM>
hipError_t adj_prep_impl(const float *d, int K, __bf16 *dA, hipStream_t s) {
    constexpr int M = MM * MM, MP = 32 * ((M + 31) / 32);
    const int Kp = (K + MF_KB - 1) / MF_KB * MF_KB;
    const long long n = (long long)Kp * MP;
    SCSC_LAUNCH(k_adj_prep_a<MM>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, K, Kp, dA);
    return hipGetLastError();
}

template <int MM>
hipError_t adjoint_dense_mfma_impl(const Geometry &g, int K, const float *r, const __bf16 *dA, float *out,
                                   hipStream_t s) {
    const int grid = persistent_grid(reinterpret_cast<const void *>(&k_adjoint_dense_mfma<MM>), TPB, 0, g.n_tiles);
    SCSC_LAUNCH(k_adjoint_dense_mfma<MM>, dim3(grid), dim3(TPB), 0, s, g.d_img, g.d_tiles, g.n_tiles, K, r,
                dA, out);
    return hipGetLastError();
}

template <int MM>
hipError_t adjoint_dense_impl(const Geometry &g, int K, const float *r, const float *d, float *out,
                              hipStream_t s) {
    constexpr int M = MM * MM, M4 = (M + 3) / 4 * 4;
    const int KC = filter_chunk<MM>();
    const int kc = K < KC ? K : KC;
    const size_t shm = (size_t)kc * M4 * sizeof(float);
    SCSC_LAUNCH(k_adjoint_dense<MM>, dim3(g.n_tiles), dim3(TPB), shm, s, g.d_img, g.d_tiles, K, r, d, out,
                KC);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_synth(const Geometry &g, int K, int m, Lists z, const float *d, const float *x,
                        const unsigned char *W, float *out, SynthMode mode, int variant, hipStream_t s) {
    SCSC_DISPATCH_M(m, synth_impl, g, K, z, d, x, W, out, mode, variant, s);
}

hipError_t launch_adjoint_shrink(const Geometry &g, int K, int m, const unsigned *mask_words,
                                 const unsigned *soff, const Pair *old_pairs, const unsigned short *old_cnt,
                                 Pair *new_pairs, unsigned short *new_cnt, const float *r, const float *d,
                                 const float *ethr, unsigned long long *nnz_acc, hipStream_t s) {
    SCSC_DISPATCH_M(m, adjoint_shrink_impl, g, K, mask_words, soff, old_pairs, old_cnt, new_pairs, new_cnt, r, d,
                    ethr, nnz_acc, s);
}

size_t adj_prep_elems(int K, int m) {
    return (size_t)((K + MF_KB - 1) / MF_KB * MF_KB) * (size_t)(32 * ((m * m + 31) / 32));
}

hipError_t launch_adj_prep(const float *d, int K, int m, __bf16 *dA, hipStream_t s) {
    SCSC_DISPATCH_M(m, adj_prep_impl, d, K, dA, s);
}

hipError_t launch_adjoint_shrink_mfma(const Geometry &g, int K, int m, const unsigned *mask_words,
                                      const unsigned *soff, const Pair *old_pairs, const unsigned short *old_cnt,
                                      Pair *new_pairs, unsigned short *new_cnt, const float *r, const __bf16 *dA,
                                      const float *ethr, unsigned long long *nnz_acc, int variant, hipStream_t s) {
    SCSC_DISPATCH_M(m, adjoint_shrink_mfma_impl, g, K, mask_words, soff, old_pairs, old_cnt, new_pairs, new_cnt, r,
                    dA, ethr, nnz_acc, variant, s);
}

hipError_t launch_adjoint_dense(const Geometry &g, int K, int m, const float *r, const float *d, float *out,
                                hipStream_t s) {
    SCSC_DISPATCH_M(m, adjoint_dense_impl, g, K, r, d, out, s);
}

hipError_t launch_adjoint_dense_mfma(const Geometry &g, int K, int m, const float *r, const __bf16 *dA, float *out,
                                     hipStream_t s) {
    SCSC_DISPATCH_M(m, adjoint_dense_mfma_impl, g, K, r, dA, out, s);
}

int persistent_grid(const void *kernel, int block_threads, size_t dyn_lds, long long items) {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            n_cu = v;
        else
            n_cu = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, dyn_lds) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    long long g = (long long)per_cu * n_cu;
    if (g > items) g = items;
    if (g >= N_XCD) g -= g % N_XCD;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace scsc
