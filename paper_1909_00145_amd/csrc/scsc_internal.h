// Internal declarations of the gfx950 stochastic-CSC library: batch geometry,
// the compact per-pixel code lists, device helpers and kernel launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "scsc.h"

namespace scsc {

// Kernel-level timing of one profiled launch scope.  While such a scope is open on
// this thread, SCSC_LAUNCH has each kernel record its own start (the scope's first
// kernel only) and end (every kernel, so the last one's end is kept) in these events
// on the launch's stream: the scope's time is then the kernels' execution from the
// first one's start to the last one's end, without the dispatch gaps around them.
struct KernelTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    bool used = false;
};
extern thread_local KernelTiming *kernel_timing;

#define SCSC_LAUNCH(kernel, grid, block, shm, stream, ...)                                            \
    do {                                                                                              \
        if (::scsc::KernelTiming *kt_ = ::scsc::kernel_timing) {                                      \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, kt_->used ? nullptr : kt_->start, \
                                  kt_->stop, 0u, __VA_ARGS__);                                        \
            kt_->used = true;                                                                         \
        } else {                                                                                      \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                        \
        }                                                                                             \
    } while (0)

// Every per-pixel kernel works on square output tiles of TS x TS pixels, one
// workgroup of TS*TS threads (4 wave64s) per tile, thread (ty, tx) <-> pixel.
constexpr int TS = 16;
constexpr int TPB = TS * TS;
constexpr int MAX_K = 1024;
constexpr int MAX_C = 5;                  // largest half-width (m = 11)
constexpr int MAX_RW = TS + 2 * MAX_C;    // side of a tile plus one filter halo
constexpr int MAX_RW2 = TS + 4 * MAX_C;   // side of a tile plus two filter halos
constexpr int TS_BIG = 32;                // synthesis tiles: TS_BIG x TS_BIG pixels, one thread each
constexpr int TPB_BIG = TS_BIG * TS_BIG;

struct ImgInfo {
    int H, W;
    long long pix_off;  // first pixel of the image in the packed pixel arrays
    int tiles_x, tiles_y;
    int tile_off;
    int index;          // image index used by the sampler
    int row_off;        // first row of the image in the global row numbering
    int pad;
};

struct TileInfo {
    int img, ty, tx, pad;
};

// One non-zero (or selected) code of a pixel: filter index and value.  The
// per-pixel lists are sorted by k and live at [off[p], off[p] + cnt[p]).
struct __align__(8) Pair {
    int k;
    float v;
};

// A per-pixel list entry tagged with its pixel column x for a pass that reads
// runs of pixels of one row: off = (x * xmul + k) * 8 modulo 2^32, the entry's
// byte offset in an LDS table with rows of xmul doubles per column.  Written
// beside the plain pairs of the non-zero lists.
struct __align__(8) XPair {
    unsigned off;
    float v;
};

// One non-zero code in the per-filter lists: position (y << 16 | x) inside its
// image, value and image.  The lists of filter k are ordered by global row
// then x and live at [fm_off[k R + r], fm_off[k R + r + 1]) for row r.
struct __align__(16) FmCode {
    unsigned yx;
    float v;
    int img;
    int pad;
};

// Device view of a batch: per-image info and the flattened tile list.
struct Geometry {
    int n_img = 0;
    int n_tiles = 0;
    long long n_pix = 0;
    int max_side = 0;
    int n_rows = 0;  // sum of image heights
    ImgInfo *d_img = nullptr;
    TileInfo *d_tiles = nullptr;
    int *d_row_img = nullptr;  // image of every global row
    int n_tiles_big = 0;             // tiles of TS_BIG x TS_BIG pixels (synthesis)
    TileInfo *d_tiles_big = nullptr;
    std::vector<TileInfo> h_tiles_big;
    std::vector<ImgInfo> h_img;
    std::vector<TileInfo> h_tiles;
};

// Compact list structure over all pixels of a batch.
struct Lists {
    const unsigned *off;       // [n_pix + 1] exclusive prefix of list capacities
    const unsigned short *cnt; // [n_pix] current list lengths
    const Pair *pairs;         // [off[n_pix]]
};

// ---- device helpers ------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
    // Philox-4x32 bijection, 10 rounds (Salmon et al., SC'11).
    const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += W0;
            k.y += W1;
        }
        unsigned hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        unsigned hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// Pixel of a 16 x 16 geometry tile owned by thread threadIdx.x of workgroup
// blockIdx.x (row-major inside the tile).
struct PixelCtx {
    TileInfo t;
    ImgInfo im;
    int ly, lx, y, x;
    bool valid;
    long long p_img;  // y * W + x
    long long gp;     // packed pixel index
};

__device__ __forceinline__ PixelCtx pixel_ctx(const ImgInfo *imgs, const TileInfo *tiles, int tile = -1) {
    PixelCtx c;
    c.t = tiles[tile < 0 ? (int)blockIdx.x : tile];
    c.im = imgs[c.t.img];
    c.ly = threadIdx.x / TS;
    c.lx = threadIdx.x % TS;
    c.y = c.t.ty * TS + c.ly;
    c.x = c.t.tx * TS + c.lx;
    c.valid = c.y < c.im.H && c.x < c.im.W;
    c.p_img = (long long)c.y * c.im.W + c.x;
    c.gp = c.im.pix_off + c.p_img;
    return c;
}

// Pixel of a flat launch over the packed pixels: thread blockIdx.x * TPB + threadIdx.x
// is packed pixel gp, so the lanes of a wave walk consecutive pixels of an image
// row (coalesced accesses to per-pixel and [K][H][W] arrays).  The image is found
// by a binary search over the images' first pixels.  Tile fields are not set.
__device__ __forceinline__ PixelCtx flat_ctx(const ImgInfo *imgs, int n_img, long long n_pix) {
    PixelCtx c;
    c.gp = (long long)blockIdx.x * TPB + threadIdx.x;
    c.valid = c.gp < n_pix;
    int lo = 0, hi = n_img - 1;
    const long long q = c.valid ? c.gp : n_pix - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].pix_off <= q) lo = mid;
        else hi = mid - 1;
    }
    c.im = imgs[lo];
    c.p_img = q - c.im.pix_off;
    c.y = (int)(c.p_img / c.im.W);
    c.x = (int)(c.p_img - (long long)c.y * c.im.W);
    c.ly = c.lx = 0;
    return c;
}
inline unsigned flat_grid(long long n_pix) { return (unsigned)((n_pix + TPB - 1) / TPB); }

// Surrogate storage: only the blocks (k, k2) with k <= k2 are kept (C_bar is
// symmetric), in row-major order of the upper triangle.
__host__ __device__ __forceinline__ long long tri_block(int k, int k2, int K) {
    return (long long)k * (2LL * K - k + 1) / 2 + (k2 - k);
}

// Work list of a persistent grid.  Hardware hands workgroup b to XCD b mod 8,
// so the workgroups of one XCD take one contiguous eighth of the work items:
// neighbouring tiles, which share halo data, are then served by the same L2.
// Items first, first + step, ... below end belong to this workgroup.
constexpr int N_XCD = 8;

// One item per workgroup, grid = xcd_grid(n): workgroup b (on XCD b % 8) takes item
// (b % 8) * (grid / 8) + b / 8, so each XCD's L2 serves a contiguous range of
// items; returns -1 for the padding workgroups.
inline unsigned xcd_grid(long long n) { return (unsigned)((n + N_XCD - 1) / N_XCD * N_XCD); }
__device__ __forceinline__ long long xcd_item(long long n) {
    const long long per = gridDim.x / N_XCD;
    const long long item = (long long)(blockIdx.x % N_XCD) * per + blockIdx.x / N_XCD;
    return item < n ? item : -1;
}
// Tile of a launch with one workgroup per tile over n tiles (any n): XCD x takes the
// x-th of eight runs of consecutive tiles (q + 1 tiles for x < n mod 8, else q, with
// q = n / 8), so the halo data that neighbouring tiles share is fetched into one L2.
// A bijection on [0, n): workgroup 8 i + x is tile start(x) + i.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b % N_XCD, i = b / N_XCD, q = n / N_XCD, r = n % N_XCD;
    return x * q + min(x, r) + i;
}
__device__ __forceinline__ void xcd_work(long long total, long long &first, long long &step, long long &end) {
    const int G = gridDim.x;
    if (G < N_XCD || G % N_XCD) {
        first = blockIdx.x;
        step = G;
        end = total;
        return;
    }
    const int x = blockIdx.x % N_XCD, slot = blockIdx.x / N_XCD;
    first = total * x / N_XCD + slot;
    step = G / N_XCD;
    end = total * (x + 1) / N_XCD;
}

// Grid of a persistent kernel: resident workgroups on the whole device (a
// multiple of 8 when possible), at most `items`.
int persistent_grid(const void *kernel, int block_threads, size_t dyn_lds, long long items);

// Matrix-core fragment types (v_mfma_f32_16x16x32_bf16 operands and result).
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float soft_threshold(float u, float t) {
    float a = fabsf(u) - t;
    return a > 0.f ? copysignf(a, u) : 0.f;
}

// Exclusive prefix sum over the TPB threads of a block.  `scratch` must hold
// TPB ints of shared memory.  Returns the thread's exclusive prefix; *total
// receives the block sum.  Contains __syncthreads.
__device__ __forceinline__ int block_exclusive_scan(int v, int *scratch, int *total) {
    const int t = threadIdx.x;
    scratch[t] = v;
    __syncthreads();
    for (int o = 1; o < TPB; o <<= 1) {
        int a = (t >= o) ? scratch[t - o] : 0;
        __syncthreads();
        scratch[t] += a;
        __syncthreads();
    }
    int incl = scratch[t];
    *total = scratch[TPB - 1];
    __syncthreads();
    return incl - v;
}

// Exclusive prefix sum over the NT threads of a block (NT a power of two).
template <int NT>
__device__ __forceinline__ int block_exclusive_scan_n(int v, int *scratch, int *total) {
    const int t = threadIdx.x;
    scratch[t] = v;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        int a = (t >= o) ? scratch[t - o] : 0;
        __syncthreads();
        scratch[t] += a;
        __syncthreads();
    }
    int incl = scratch[t];
    *total = scratch[NT - 1];
    __syncthreads();
    return incl - v;
}

// ---- launchers (host) ----------------------------------------------------
// All launchers return hipSuccess or the launch error.

// mask_words[w][p] bit b <=> coordinate k = 32 w + b of pixel p is selected;
// cnt[p] = number of selected coordinates of pixel p.
hipError_t launch_mask_count(const Geometry &g, int K, unsigned long long thr, unsigned long long seed,
                             unsigned draw, unsigned *mask_words, unsigned *cnt, hipStream_t s);
// Exclusive prefix of cnt[0..n) into off[0..n]; off[n] = low 32 bits of the total,
// total64 (device) = the exact total.  tmp needs scan_tmp_elems(n) u64.
long long scan_tmp_elems(long long n);
hipError_t launch_scan(const unsigned *cnt, unsigned *off, long long n, unsigned long long *tmp,
                       unsigned long long *total64, hipStream_t s);
// Warm start: list of non-zero selected codes of z_prev (eq. 4 restricted to S).
// nnz_acc (device, may be null) accumulates the number of non-zeros written.
hipError_t launch_gather_selected(const Geometry &g, int K, const unsigned *mask_words, const unsigned *soff,
                                  const float *z, Pair *pairs, unsigned short *cnt, unsigned long long *nnz_acc,
                                  hipStream_t s);
// Mode of the synthesis kernel.
enum SynthMode { SYNTH_RESIDUAL = 0, SYNTH_PLAIN = 1, SYNTH_WEIGHTED = 2 };
// out = W (x - D z) (RESIDUAL), D z (PLAIN) or W (D z) (WEIGHTED); z given as lists.
// variant (identical results): 0: 16x16 tiles, 1 thread per output pixel; 1: 16x16, 4 threads;
// 2: 16x8, 2 threads; 3: 16x8, 4 threads.
hipError_t launch_synth(const Geometry &g, int K, int m, Lists z, const float *d, const float *x,
                        const unsigned char *W, float *out, SynthMode mode, int variant, hipStream_t s);
// One proximal-gradient iteration on the selected coordinates (FP32 VALU).
// BF16 operands on the matrix cores, FP32 accumulation; same lists and epilogue.
// The filters enter as dA, written by launch_adj_prep (adj_prep_elems(K, m) elements).
size_t adj_prep_elems(int K, int m);
hipError_t launch_adj_prep(const float *d, int K, int m, __bf16 *dA, hipStream_t s);
// variant 0: the next chunk's operands load during the current chunk (two
// workgroups per CU); 1: at the chunk's start (three per CU).  Same bits.
// nnz_acc may be null (the count of non-zeros is then not added).
hipError_t launch_adjoint_shrink_mfma(const Geometry &g, int K, int m, const unsigned *mask_words,
                                      const unsigned *soff, const Pair *old_pairs, const unsigned short *old_cnt,
                                      Pair *new_pairs, unsigned short *new_cnt, const float *r, const __bf16 *dA,
                                      const float *ethr, unsigned long long *nnz_acc, int variant, hipStream_t s);
hipError_t launch_adjoint_shrink(const Geometry &g, int K, int m, const unsigned *mask_words,
                                 const unsigned *soff, const Pair *old_pairs, const unsigned short *old_cnt,
                                 Pair *new_pairs, unsigned short *new_cnt, const float *r, const float *d,
                                 const float *ethr, unsigned long long *nnz_acc, hipStream_t s);
// Dense codes from lists (zeros elsewhere).
hipError_t launch_scatter_dense(const Geometry &g, int K, Lists z, float *zout, hipStream_t s);
// Lists of the non-zero codes of a dense z: count, then fill.
hipError_t launch_count_nonzero(const Geometry &g, int K, const float *z, unsigned *cnt, hipStream_t s);
// xp (may be null): the same entries tagged with their columns for row stride xmul.
hipError_t launch_fill_nonzero(const Geometry &g, int K, const float *z, const unsigned *off, Pair *pairs,
                               unsigned short *cnt, XPair *xp, unsigned xmul, hipStream_t s);
// Exact-capacity lists from a code step's lists (lengths in.cnt at offsets in.off):
// launch_counts_u32 widens the lengths for launch_scan, whose offsets off feed
// launch_compact_lists (entries, lengths and, with xp, the tags of launch_fill_nonzero).
hipError_t launch_counts_u32(const unsigned short *cnt, long long n, unsigned *out, hipStream_t s);
hipError_t launch_compact_lists(const Geometry &g, Lists in, const unsigned *off, Pair *pairs, unsigned short *cnt,
                                XPair *xp, unsigned xmul, hipStream_t s);
// Held codes: lists of the non-zero codes of z off the sample (count, then fill),
// and the scatter of the sample only (the other coordinates of z unchanged).
hipError_t launch_count_held(const Geometry &g, int K, const unsigned *mask_words, const float *z, unsigned *cnt,
                             hipStream_t s);
hipError_t launch_fill_held(const Geometry &g, int K, const unsigned *mask_words, const float *z, const unsigned *off,
                            Pair *pairs, unsigned short *cnt, hipStream_t s);
hipError_t launch_scatter_selected(const Geometry &g, int K, const unsigned *mask_words, Lists zl, float *z,
                                   hipStream_t s);
// ADMM code solver on the sample (kernels_admm.hip).  S-vectors are FP32 over the
// selected coordinates at [soff[p], soff[p + 1]), filters ascending per pixel.
hipError_t launch_sel_list(const Geometry &g, int K, const unsigned *mask_words, const unsigned *soff, const float *z,
                           Pair *pairs, unsigned short *cnt, hipStream_t s);
hipError_t launch_pack(const Pair *sel, const float *val, Pair *pairs, long long n, hipStream_t s);
hipError_t launch_unpack(const Geometry &g, const unsigned *soff, const Pair *sel, const Pair *cl,
                         const unsigned short *ccnt, float *out, hipStream_t s);
// Per-image segments seg[n_img + 1] of the S-vectors, and the segmented CG:
// dot products into the scalars scs[n] = {rr, alpha, beta} of image n (mode 0
// sets rr, mode 1 alpha = rr / dot, mode 2 beta = dot / rr and rr = dot);
// part holds admm_dot_elems(n_img) doubles.
long long admm_dot_elems(int n_img);
hipError_t launch_seg(const Geometry &g, const unsigned *soff, unsigned *seg, hipStream_t s);
hipError_t launch_cg_dot(const Geometry &g, const float *a, const float *b, const unsigned *seg, double *part,
                         int mode, double *scs, hipStream_t s);
hipError_t launch_axpy_alpha(const Geometry &g, float *y, const float *x, const double *scs, const unsigned *seg,
                             float sgn, hipStream_t s);
hipError_t launch_cg_dir(const Geometry &g, float *q, const float *r, const double *scs, const unsigned *seg,
                         hipStream_t s);
hipError_t launch_add_scaled(float *Aq, const float *q, float rho, long long n, hipStream_t s);
hipError_t launch_cg_init(float *r, float *q, const float *b0, const float *v, const float *u, const float *Aq,
                          float rho, long long n, hipStream_t s);
hipError_t launch_admm_update(const float *zt, float *v, float *u, float alpha, float thr, long long n,
                              hipStream_t s);
hipError_t launch_count_nz(const float *v, long long n, unsigned long long *out, hipStream_t s);
// Selection bytes (csc_mask).
hipError_t launch_expand_mask(const Geometry &g, int K, const unsigned *mask_words, unsigned char *mask,
                              hipStream_t s);
// Sum of cnt over all pixels into *out (device u64).
hipError_t launch_sum_counts(const unsigned short *cnt, long long n, unsigned long long *out, hipStream_t s);

// Filter-major correlation from the per-filter lists: partial[c][k][t] over
// chunk c of filter k's codes (corr_chunks(K) chunks), FP64 accumulation.
int corr_chunks(int K);
hipError_t launch_corr_fm(const Geometry &g, int K, int m, const unsigned *fm_off, const FmCode *fm, const float *r,
                          const unsigned char *W, bool weight_rhs, double *partial, hipStream_t s);
hipError_t launch_reduce_partials_f64_to_f32(const double *partial, int nblocks, int n, float *out, hipStream_t s);
hipError_t launch_reduce_partials_f64_add(const double *partial, int nblocks, int n, double *inout,
                                          hipStream_t s);
// Dense adjoint D^T r (every coordinate).
hipError_t launch_adjoint_dense(const Geometry &g, int K, int m, const float *r, const float *d, float *out,
                                hipStream_t s);
// The same with BF16 operands on the matrix cores (FP32 accumulation); the filters
// enter as dA, written by launch_adj_prep (adj_prep_elems(K, m) elements).
hipError_t launch_adjoint_dense_mfma(const Geometry &g, int K, int m, const float *r, const __bf16 *dA, float *out,
                                     hipStream_t s);

// Filter updates.
hipError_t launch_fill(float *v, int n, float val, hipStream_t s);
// Power-iteration step: lam = <v, w>, v = w / ||w|| (kept when w = 0, lam = 0).
hipError_t launch_power_update(float *v, const float *w, int n, double *lam, hipStream_t s);
// d_k <- P(d_k + G_k / lam) (lam <= 0: P(d_k)).
hipError_t launch_batch_update(float *d, const float *G, const double *lam, int K, int M, hipStream_t s);
// d_k <- P(d_k - (y_k - B_k) / Ld_sum).
hipError_t launch_online_update(float *d, const double *y, const double *B, double Ld_sum, int K, int M,
                                hipStream_t s);
// Surrogates (lag layout).  Per-filter row lists of the non-zero codes (from
// exact-capacity lists), C += sum Z^T W Z by owner blocks, and y = C d.
hipError_t launch_fm_lists(const Geometry &g, int K, Lists z, unsigned *fm_cnt, unsigned *fm_off, FmCode *fm,
                           unsigned long long *scan_tmp, unsigned long long *total64, hipStream_t s);
hipError_t launch_surrogate_blocks(const Geometry &g, int K, int m, const unsigned *fm_off, const FmCode *fm,
                                   const unsigned char *W, double *C, hipStream_t s);
// Unmasked case: lag sums Rl[lag][k][k2] (surrogate_lag_elems doubles), band sums
// Es[4 c][lag][k][k2] (k <= k2; skipped when Es is null), expansion, corners.
// part: surrogate_lag_part_elems doubles of workspace (per-chunk partial sums).
// With xp (the entries of z tagged for row stride lag_rows_stride) and the
// per-filter lists, the lags delta >= 0 are summed by filter-major runs, else by
// pixel slots.  sums_done (may be null) is recorded on s once R is formed, before
// the band sums.
long long surrogate_lag_elems(int K, int m);
long long surrogate_lag_part_elems(const Geometry &g, int K, int m);
unsigned lag_rows_stride(const Geometry &g, int K, int m);  // 0: the run pass does not apply
hipError_t launch_surrogate_lag(const Geometry &g, int K, int m, Lists z, const XPair *xp, const unsigned *fm_off,
                                const FmCode *fm, double *part, double *Rl, double *Es, hipEvent_t sums_done,
                                hipStream_t s);
// Power iteration on the zero-padded normal matrix given by the lag sums.
// Rf = the lag sums rounded to FP32 (a step-size estimate needs no more), in
// [k][k2][lag] order (launch_lag_to_f32).  The matvec multiplies v = w / ||w||,
// ||w||^2 = sum of nparts[0, n_nparts), and writes part[lag_matvec_chunks(K)][K][m*m]
// FP64 partial sums; launch_power_reduce sums them into the next w (FP32) with
// power_reduce_blocks(n) partials of ||w||^2 and v . w; launch_power_final sets
// lam = v . w of the last product.
int lag_matvec_chunks(int K);
hipError_t launch_lag_to_f32(int K, int m, const double *Rl, float *Rf, hipStream_t s);
hipError_t launch_lag_matvec(int K, int m, const float *Rf, const float *w, const double *nparts, int n_nparts,
                             double *part, hipStream_t s);
int power_reduce_blocks(int n);
hipError_t launch_power_reduce(const double *part, int nch, int n, float *w_out, const float *w_prev,
                               const double *nparts_prev, int n_nparts, double *nparts_out, double *dparts_out,
                               hipStream_t s);
hipError_t launch_power_start(double *nparts, int nb, double nn0, hipStream_t s);
hipError_t launch_power_final(const double *nparts, const double *dparts, int nb, double *lam, hipStream_t s);
// C_bar += R - band terms for the stored blocks; with d non-null also y = C_bar d of
// the updated C_bar (part: surrogate_matvec_partial_elems doubles).  The corner
// correction must already be in C_bar.
hipError_t launch_surrogate_expand(int K, int m, const double *Rl, const double *Es, unsigned short *tab, double *C,
                                   const float *d, double *part, double *y, hipStream_t s);
hipError_t launch_surrogate_corner(const Geometry &g, int K, int m, Lists z, double *C, hipStream_t s);
hipError_t launch_surrogate_matvec(int K, int m, const double *C, const float *d, double *partial, double *y,
                                   hipStream_t s);
long long surrogate_matvec_partial_elems(int K, int m);

// G = sum_i Z_i^T r_i ([K][m][m], FP32) on the matrix cores from per-pixel code lists,
// BF16 operands, FP32 accumulation; part needs corr_mfma_blocks(g, K) * K * m^2 floats.
int corr_mfma_blocks(const Geometry &g, int K);
// out = W (x - D z) / D z / W (D z) (mode as launch_synth) with BF16 operands on the
// matrix cores and FP32 accumulation.  The filters enter as dA, the BF16 operand
// written by launch_synth_mfma_prep (synth_mfma_prep_elems(K) elements).
size_t synth_mfma_prep_elems(int K);
hipError_t launch_synth_mfma_prep(const float *d, int K, int m, __bf16 *dA, hipStream_t s);
// variant 0: 16 filters per LDS chunk, 1: 32, 2: 8 (four workgroups per CU).  Same bits.
constexpr int SYNTH_MFMA_VARIANTS = 3;
hipError_t launch_synth_mfma(const Geometry &g, int K, int m, Lists z, const __bf16 *dA, const float *x,
                             const unsigned char *W, float *out, int mode, int variant, hipStream_t s);
hipError_t launch_corr_mfma(const Geometry &g, int K, int m, Lists z, const float *r, float *part, float *G,
                            hipStream_t s);

// Unrolled-layer elementwise kernels over n dense code entries:
// out = mask ? shrink(z + eta g, thr) : 0;  gu = (mask && |z + eta g| > thr) ? gout : 0;
// out = a x + b y (y may be null: out = a x).
hipError_t launch_ista_update(long long n, const float *z, const float *g, const unsigned char *mask, float eta,
                              float thr, float *out, hipStream_t s);
hipError_t launch_ista_grad_u(long long n, const float *z, const float *g, const unsigned char *mask,
                              const float *gout, float eta, float thr, float *gu, hipStream_t s);
hipError_t launch_axpby(long long n, float a, const float *x, float b, const float *y, float *out, hipStream_t s);
// dst[0] = a, dst[1] = b (device scalars written in stream order).
hipError_t launch_set2(float *dst, float a, float b, hipStream_t s);
hipError_t launch_set_step(float *dst, const double *L, double step, double lambda, unsigned long long *counter,
                           hipStream_t s);

// FP64 objective: out[0] = data term, out[1] = L1 norm.
hipError_t launch_objective(const Geometry &g, int K, int m, const float *x, const unsigned char *W,
                            const float *d, const float *z, double *partial, double *out, hipStream_t s);
// FP64 Lipschitz bound of the code gradient.
hipError_t launch_lipschitz_code(const float *d, int K, int m, int P, double *tmp, double *out, hipStream_t s);
long long lipschitz_tmp_elems(int K, int m, int P);

}  // namespace scsc
