// Online surrogate kernels for gfx950 (the surrogates of eq. (8) and the
// gradient of the surrogate problem, eq. (9)), FP64:
//   C_bar += sum_n Z_n^T W_n Z_n   and   y = C_bar d.
//
// Entry ((k, s), (k2, s2)) of Z^T W Z is sum_p W[p] z_k[p - s] z_k2[p - s2], p over
// the image.  With z zero outside the image and no observation mask it equals
//     R(delta) - E(delta, s),      delta = s - s2,
// where R(delta) = sum_q z_k[q] z_k2[q + delta] sums every pair of codes at lag
// delta, and E sums the same products over the output pixels p outside the
// image (a ring of width c).  Splitting the ring into its top and bottom rows
// (all columns) and left and right columns (all rows) double counts its four
// c x c corners, so
//     E = E_top(delta, s_y) + E_bottom(delta, s_y) + E_left(delta, s_x)
//         + E_right(delta, s_x) - E_corners(delta, s),
// and each side term is a prefix sum over the first (last) c rows (columns) of
// the image of the lag sums restricted to codes in that row (column).  The lag
// sums come from filter-major runs of non-zero codes: a workgroup owns a
// tap-row offset, a few filters k and a range of image rows, keeps the sums
// for every column offset and partner filter in LDS, and pairs each of its
// codes with the contiguous run of partner codes in the row below; the corner
// term is formed exactly from the corner ring pixels.
// With an observation mask the masked pixels are excluded as well; that case
// uses a tiled kernel that enumerates every excluded pixel.
#include "scsc_internal.h"

namespace scsc {

namespace {

__host__ __device__ __forceinline__ int lagp(int a, int m) {
    // sum_{b = -(m-1)}^{a-1} (m - |b|)
    if (a <= 0) return (m + a - 1) * (m + a) / 2;
    return m * (m - 1) / 2 + a * m - a * (a - 1) / 2;
}

// ---- per-filter row lists ---------------------------------------------------
// fm_cnt[k * R + r] = number of non-zero codes of filter k in global row r.
__global__ __launch_bounds__(256) void k_fm_count(const ImgInfo *imgs, const int *row_img, Lists zl, int R, int K,
                                                  unsigned *fm_cnt) {
    extern __shared__ unsigned cntk[];  // [K]
    const int r = blockIdx.x;
    const ImgInfo im = imgs[row_img[r]];
    const int y = r - im.row_off;
    const long long gp0 = im.pix_off + (long long)y * im.W;
    for (int k = threadIdx.x; k < K; k += 256) cntk[k] = 0u;
    __syncthreads();
    for (int x = threadIdx.x; x < im.W; x += 256) {
        const long long gp = gp0 + x;
        const unsigned o = zl.off[gp];
        const int n = zl.cnt[gp];
        for (int j = 0; j < n; ++j) atomicAdd(&cntk[zl.pairs[o + j].k], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += 256) fm_cnt[(long long)k * R + r] = cntk[k];
}

constexpr int FM_CAP = 4096;
constexpr int FM_BM_BYTES = 48 * 1024;  // LDS for the per-filter occupancy bitmaps of one row

// Row r's entries, regrouped by filter in x order: fm[fm_off[k * R + r] + j] = (y << 16 | x, v).
// With bitmaps (nww 64-bit words per filter, nww > 0): bit x of filter k's bitmap
// marks pixel x holding a code of k, and an entry's slot is the number of set
// bits below x (its rank among the row's codes of k in x order).  Otherwise each
// filter scans the row's entries.  Requires the pixel lists of the row to be
// contiguous (exact-capacity lists).
__global__ __launch_bounds__(256) void k_fm_fill(const ImgInfo *imgs, const int *row_img, Lists zl, int R, int K,
                                                 int nww, const unsigned *fm_off, FmCode *fm) {
    extern __shared__ unsigned long long bm[];  // [K][nww] when nww > 0
    __shared__ Pair ent[FM_CAP];
    __shared__ unsigned short ex[FM_CAP];
    const int r = blockIdx.x;
    const int img = row_img[r];
    const ImgInfo im = imgs[img];
    const int y = r - im.row_off;
    const long long gp0 = im.pix_off + (long long)y * im.W;
    if (nww > 0) {
        for (int i = threadIdx.x; i < K * nww; i += 256) bm[i] = 0ull;
        __syncthreads();
        for (int x = threadIdx.x; x < im.W; x += 256) {
            const long long gp = gp0 + x;
            const unsigned o = zl.off[gp];
            const int n = zl.cnt[gp];
            for (int j = 0; j < n; ++j)
                atomicOr(&bm[(long long)zl.pairs[o + j].k * nww + (x >> 6)], 1ull << (x & 63));
        }
        __syncthreads();
        for (int x = threadIdx.x; x < im.W; x += 256) {
            const long long gp = gp0 + x;
            const unsigned o = zl.off[gp];
            const int n = zl.cnt[gp];
            for (int j = 0; j < n; ++j) {
                const Pair p = zl.pairs[o + j];
                const unsigned long long *row = bm + (long long)p.k * nww;
                unsigned rank = __popcll(row[x >> 6] & ((1ull << (x & 63)) - 1ull));
                for (int w = 0; w < (x >> 6); ++w) rank += __popcll(row[w]);
                fm[fm_off[(long long)p.k * R + r] + rank] = FmCode{((unsigned)y << 16) | (unsigned)x, p.v, img, 0};
            }
        }
        return;
    }
    const unsigned base = zl.off[gp0];
    const unsigned total = zl.off[gp0 + im.W] - base;
    const bool staged = total <= FM_CAP;
    if (staged) {
        for (int x = threadIdx.x; x < im.W; x += 256) {
            const long long gp = gp0 + x;
            const unsigned o = zl.off[gp];
            const int n = zl.cnt[gp];
            for (int j = 0; j < n; ++j) {
                ent[o - base + j] = zl.pairs[o + j];
                ex[o - base + j] = (unsigned short)x;
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += 256) {
        unsigned w = fm_off[(long long)k * R + r];
        if (staged) {
            for (unsigned e = 0; e < total; ++e) {
                const Pair p = ent[e];
                if (p.k == k) fm[w++] = FmCode{((unsigned)y << 16) | ex[e], p.v, img, 0};
            }
        } else {
            for (int x = 0; x < im.W; ++x) {
                const long long gp = gp0 + x;
                const unsigned o = zl.off[gp];
                const int n = zl.cnt[gp];
                for (int j = 0; j < n; ++j) {
                    const Pair p = zl.pairs[o + j];
                    if (p.k == k) fm[w++] = FmCode{((unsigned)y << 16) | (unsigned)x, p.v, img, 0};
                }
            }
        }
    }
}

// ---- block accumulation -----------------------------------------------------
// With z zero outside the image, entry ((k, s), (k2, s2)) of the batch term is
//     R(delta) - E(delta, s),   delta = s - s2,
// where R(delta) = sum_q z_k[q] z_k2[q + delta] is the full-lag sum over every
// pair of codes, and E(delta, s) = sum_{p excluded} z_k[p - s] z_k2[p - s2] runs
// over the output pixels the objective does not contain: the ring of width c
// around the image and, with an observation mask, the masked pixels.  Both are
// accumulated per image tile of SB_TQ x SB_TQ code positions from dense planes
// of the two filters' codes on the tile grown by 2c, with per-row occupancy
// bitmasks to enumerate partners.  Every pair costs one FP64 LDS atomic.
constexpr int SB_THREADS = 512;
constexpr int SB_TQ = 32;

template <int MM>
__global__ __launch_bounds__(SB_THREADS) void k_sur_block(const ImgInfo *imgs, int n_img, int K, int R,
                                                          const unsigned *__restrict__ fm_off,
                                                          const FmCode *__restrict__ fm,
                                                          const unsigned char *__restrict__ W,
                                                          double *__restrict__ Cbar) {
    constexpr int C = MM / 2, M = MM * MM, M2 = M * M, L = 2 * MM - 1;
    constexpr int PW = SB_TQ + 4 * C;  // region side (<= 64: one 64-bit mask per row)
    constexpr int XW = SB_TQ + 2 * C;  // side of the tile grown by c
    static_assert(PW <= 64, "region rows must fit a 64-bit mask");
    __shared__ double Cb[M2];                    // -E, lag layout
    __shared__ double Rb[L * L];                 // R per lag
    __shared__ float pl[2][PW * PW];             // code planes of k and k2 on the region
    __shared__ unsigned long long bm[2][PW];     // row occupancy of the planes
    __shared__ unsigned short el[SB_TQ * SB_TQ]; // codes of k inside the tile (region index)
    __shared__ int nel;
    const int k = blockIdx.y, k2 = blockIdx.x;
    if (k2 < k) return;
    for (int i = threadIdx.x; i < M2; i += SB_THREADS) Cb[i] = 0.0;
    for (int i = threadIdx.x; i < L * L; i += SB_THREADS) Rb[i] = 0.0;
    const int f2[2] = {k, k2};
    for (int n = 0; n < n_img; ++n) {
        const ImgInfo im = imgs[n];
        const unsigned a = fm_off[(long long)k * R + im.row_off];
        const unsigned b = fm_off[(long long)k * R + im.row_off + im.H];
        const unsigned a2 = fm_off[(long long)k2 * R + im.row_off];
        const unsigned b2 = fm_off[(long long)k2 * R + im.row_off + im.H];
        if (a == b || a2 == b2) continue;  // no pair in this image
        for (int y0 = 0; y0 < im.H; y0 += SB_TQ) {
            for (int x0 = 0; x0 < im.W; x0 += SB_TQ) {
                const int ry0 = y0 - 2 * C, rx0 = x0 - 2 * C;  // region origin
                __syncthreads();
                for (int i = threadIdx.x; i < 2 * PW * PW; i += SB_THREADS) (&pl[0][0])[i] = 0.f;
                if (threadIdx.x < 2 * PW) (&bm[0][0])[threadIdx.x] = 0ull;
                if (threadIdx.x == 0) nel = 0;
                __syncthreads();
                // planes: one thread per (filter, region row) scans that row's list
                if (threadIdx.x < 2 * PW) {
                    const int f = threadIdx.x / PW, rr = threadIdx.x % PW;
                    const int gy = ry0 + rr;
                    if (gy >= 0 && gy < im.H) {
                        const long long row = (long long)f2[f] * R + im.row_off + gy;
                        const unsigned j1 = fm_off[row + 1];
                        unsigned long long bits = 0;
                        for (unsigned j = fm_off[row]; j < j1; ++j) {
                            const FmCode e = fm[j];
                            const int c = (int)(e.yx & 0xFFFFu) - rx0;
                            if (c < 0) continue;
                            if (c >= PW) break;
                            pl[f][rr * PW + c] = e.v;
                            bits |= 1ull << c;
                        }
                        bm[f][rr] = bits;
                    }
                }
                __syncthreads();
                // codes of k inside the tile
                if (threadIdx.x < SB_TQ) {
                    const int rr = 2 * C + threadIdx.x;
                    unsigned long long bits = (bm[0][rr] >> (2 * C)) & ((1ull << SB_TQ) - 1ull);
                    if (bits) {
                        int pos = atomicAdd(&nel, __popcll(bits));
                        while (bits) {
                            const int c = __ffsll((long long)bits) - 1;
                            bits &= bits - 1ull;
                            el[pos++] = (unsigned short)(rr * PW + 2 * C + c);
                        }
                    }
                }
                __syncthreads();
                // R: every pair (q in tile, q + delta anywhere)
                for (int e = threadIdx.x; e < nel; e += SB_THREADS) {
                    const int ri = el[e];
                    const int ry = ri / PW, rx = ri % PW;
                    const double v = (double)pl[0][ri];
#pragma unroll
                    for (int dy = -2 * C; dy <= 2 * C; ++dy) {
                        unsigned long long bits = (bm[1][ry + dy] >> (rx - 2 * C)) & ((1ull << L) - 1ull);
                        while (bits) {
                            const int bx = __ffsll((long long)bits) - 1;
                            bits &= bits - 1ull;
                            const double v2 = (double)pl[1][(ry + dy) * PW + rx - 2 * C + bx];
                            atomicAdd(&Rb[(dy + 2 * C) * L + bx], v * v2);
                        }
                    }
                }
                // E: excluded output pixels owned by this tile (ring pixels whose
                // clamped position lies in the tile; masked pixels of the tile)
                for (int idx = threadIdx.x; idx < XW * XW; idx += SB_THREADS) {
                    const int py_r = C + idx / XW, px_r = C + idx % XW;
                    const int py = ry0 + py_r, px = rx0 + px_r;
                    const bool inside = py >= 0 && py < im.H && px >= 0 && px < im.W;
                    bool excluded;
                    if (inside) {
                        excluded = W && py >= y0 && py < y0 + SB_TQ && px >= x0 && px < x0 + SB_TQ &&
                                   !W[im.pix_off + (long long)py * im.W + px];
                    } else {
                        const int cy = min(max(py, 0), im.H - 1), cx = min(max(px, 0), im.W - 1);
                        excluded = cy >= y0 && cy < y0 + SB_TQ && cx >= x0 && cx < x0 + SB_TQ &&
                                   py >= -C && py < im.H + C && px >= -C && px < im.W + C;
                    }
                    if (!excluded) continue;
                    // codes of k and k2 in the window p + [-c, c]^2
                    for (int wa = -C; wa <= C; ++wa) {
                        unsigned long long ba = (bm[0][py_r + wa] >> (px_r - C)) & ((1ull << MM) - 1ull);
                        while (ba) {
                            const int ca = __ffsll((long long)ba) - 1;
                            ba &= ba - 1ull;
                            // code a at region (py_r + wa, px_r - C + ca): s = p - q_a
                            const int sy = -wa, sx = C - ca;
                            const double va = (double)pl[0][(py_r + wa) * PW + px_r - C + ca];
                            for (int wb = -C; wb <= C; ++wb) {
                                unsigned long long bb = (bm[1][py_r + wb] >> (px_r - C)) & ((1ull << MM) - 1ull);
                                while (bb) {
                                    const int cb = __ffsll((long long)bb) - 1;
                                    bb &= bb - 1ull;
                                    const int sy2 = -wb, sx2 = C - cb;
                                    const double vb = (double)pl[1][(py_r + wb) * PW + px_r - C + cb];
                                    const int dy = sy - sy2, dx = sx - sx2;
                                    const int wx = MM - (dx < 0 ? -dx : dx);
                                    const int sylo = max(-C, dy - C), sxlo = max(-C, dx - C);
                                    const int wy = MM - (dy < 0 ? -dy : dy);
                                    const int off = lagp(dy, MM) * M + wy * lagp(dx, MM);
                                    atomicAdd(&Cb[off + (sy - sylo) * wx + (sx - sxlo)], -va * vb);
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // C_bar(k, k2) += R + (-E) (upper-triangle block storage)
    double *blk = Cbar + tri_block(k, k2, K) * M2;
    const int slot = threadIdx.x / 128, t = threadIdx.x % 128;
    for (int di = slot; di < L * L; di += SB_THREADS / 128) {
        const int dy = di / L - (MM - 1), dx = di % L - (MM - 1);
        const int wy = MM - (dy < 0 ? -dy : dy), wx = MM - (dx < 0 ? -dx : dx);
        if (t >= wy * wx) continue;
        const int off = lagp(dy, MM) * M + wy * lagp(dx, MM);
        blk[off + t] += Cb[off + t] + Rb[di];
    }
}

// Lag-layout position table: tab[i] = lag index * 128 + position inside the lag's run.
template <int MM>
__global__ void k_lag_table(unsigned short *tab) {
    constexpr int M = MM * MM, L = 2 * MM - 1, LL = L * L;
    const int di = blockIdx.x * blockDim.x + threadIdx.x;
    if (di >= LL) return;
    const int dy = di / L - (MM - 1), dx = di % L - (MM - 1);
    const int wy = MM - (dy < 0 ? -dy : dy), wx = MM - (dx < 0 ? -dx : dx);
    const int off = lagp(dy, MM) * M + wy * lagp(dx, MM);
    for (int t = 0; t < wy * wx; ++t) tab[off + t] = (unsigned short)(di * 128 + t);
}

// Lag-major accumulation: workgroup (lag delta, chunk of first filters, pixel
// chunk or band class) owns the K x K matrix R_delta[k][k2] = sum_q z_k[q]
// z_k2[q + delta] in LDS and adds the outer products of the code lists of every
// pixel pair (q, q + delta) of its pixel set.
//   band == 0: every pixel of the batch, split into gridDim.z chunks; lags delta >= 0
//     only, since R_{-delta} = R_delta^T; chunk z writes its partial sums to
//     out[z][delta][k][k2] (coalesced), and k_lag_sum adds the chunks and forms both
//     halves of Rl[lag][k][k2].
//   band == 1: blockIdx.z = side * c + j selects row (column) j of the top, bottom,
//     left or right band of every image; every lag; stored into Es[cls][lag][k][k2]
//     (k <= k2).
constexpr int LO_THREADS = 1024;
constexpr int LO_U = 8;  // list entries per pixel held in registers

template <int MM>
__global__ __launch_bounds__(LO_THREADS, 8) void k_lag_outer(const ImgInfo *imgs, int n_img, long long n_pix,
                                                          int max_side, int K, Lists zl, int band, int KC,
                                                          double *__restrict__ out) {
    constexpr int C = MM / 2, L = 2 * MM - 1, LL = L * L;
    constexpr int NC = C > 0 ? C : 1;
    extern __shared__ double Rd[];  // [KC][K]
    // band: blockIdx.x = t L + e takes the t-th of the c offsets dlt in (j - c, j] across
    // the band (the only ones whose band row j is read and can be non-zero) and the
    // e-th along it
    int di;
    if (band) {
        const int sd = (int)blockIdx.z / NC, jj = (int)blockIdx.z % NC;
        const int t = (int)blockIdx.x / L, e = (int)blockIdx.x % L - 2 * C;
        const int dl = jj - C + 1 + t;
        const int dyb = sd == 0 ? -dl : sd == 1 ? dl : e, dxb = sd == 2 ? -dl : sd == 3 ? dl : e;
        di = (dyb + 2 * C) * L + dxb + 2 * C;
    } else {
        di = (LL - 1) / 2 + (int)blockIdx.x;
    }
    const int dy = di / L - 2 * C, dx = di % L - 2 * C;
    if (band) {
        // The expansion uses band row j of a side only where it lies inside the
        // strip cut off by some tap offset of this lag: j < min(c, c -+ delta).
        const int sd = (int)blockIdx.z / NC, jj = (int)blockIdx.z % NC;
        const int dlt = sd == 0 ? -dy : sd == 1 ? dy : sd == 2 ? -dx : dx;
        // never read: band rows j >= min(c, c + dlt); identically zero (the partner
        // pixel lies outside every image): dlt > j; the expansion takes those as 0
        if (jj >= min(C, C + dlt) || dlt > jj) return;
    }
    const int klo = blockIdx.y * KC, khi = min(K, klo + KC);
    for (int i = threadIdx.x; i < KC * K; i += LO_THREADS) Rd[i] = 0.0;
    __syncthreads();
    const int cls = band ? (int)blockIdx.z : -1;
    const int side = band ? cls / NC : -1, j = band ? cls % NC : 0;
    // band == 0: a chunk of the packed pixels; band == 1: slot (image n, position)
    // of a flat range over all images, so every image's band row is in flight at once
    const long long chunk = band ? 0 : (n_pix + gridDim.z - 1) / gridDim.z;
    const long long plo = band ? 0 : chunk * blockIdx.z, phi = band ? (long long)n_img * max_side : min(n_pix, plo + chunk);
    int n = 0;
    ImgInfo im = imgs[0];
    long long iend = (long long)im.H * im.W;
    {
        for (long long t = plo + threadIdx.x; t < phi; t += LO_THREADS) {
            int y, x;
            if (!band) {
                while (t >= iend) {  // advance to the image holding packed pixel t
                    im = imgs[++n];
                    iend = im.pix_off + (long long)im.H * im.W;
                }
                const unsigned pi = (unsigned)(t - im.pix_off);  // < 2^31
                y = (int)(pi / (unsigned)im.W);
                x = (int)(pi - (unsigned)y * (unsigned)im.W);
            } else {
                int nn, pos;
                if (phi < (1LL << 31)) {  // uniform: 32-bit division
                    nn = (int)((unsigned)t / (unsigned)max_side);
                    pos = (int)((unsigned)t - (unsigned)nn * (unsigned)max_side);
                } else {
                    nn = (int)(t / max_side);
                    pos = (int)(t % max_side);
                }
                if (nn != n || t == threadIdx.x) {
                    n = nn;
                    im = imgs[n];
                }
                const int len = side < 2 ? im.W : im.H, across = side < 2 ? im.H : im.W;
                if (pos >= len || j >= across) continue;
                if (side == 0) {
                    y = j;
                    x = pos;
                } else if (side == 1) {
                    y = im.H - 1 - j;
                    x = pos;
                } else if (side == 2) {
                    y = pos;
                    x = j;
                } else {
                    y = pos;
                    x = im.W - 1 - j;
                }
            }
            const int y2 = y + dy, x2 = x + dx;
            if (y2 < 0 || y2 >= im.H || x2 < 0 || x2 >= im.W) continue;
            const long long gp = im.pix_off + (long long)y * im.W + x;
            const int ca = zl.cnt[gp];
            if (ca == 0) continue;
            const long long gp2 = im.pix_off + (long long)y2 * im.W + x2;
            const int cb = zl.cnt[gp2];
            if (cb == 0) continue;
            const unsigned oa = zl.off[gp], ob = zl.off[gp2];
            // the first LO_U codes of both lists are loaded together into registers
            Pair A[LO_U], B[LO_U];
#pragma unroll
            for (int u = 0; u < LO_U; ++u) {
                if (u < ca) A[u] = zl.pairs[oa + u];
                if (u < cb) B[u] = zl.pairs[ob + u];
            }
#pragma unroll
            for (int u = 0; u < LO_U; ++u) {
                if (u >= ca || A[u].k < klo || A[u].k >= khi) continue;
                double *row = Rd + (long long)(A[u].k - klo) * K;
                const double va = (double)A[u].v;
#pragma unroll
                for (int w = 0; w < LO_U; ++w)
                    if (w < cb) atomicAdd(row + B[w].k, va * (double)B[w].v);
                for (int w = LO_U; w < cb; ++w) {
                    const Pair eb = zl.pairs[ob + w];
                    atomicAdd(row + eb.k, va * (double)eb.v);
                }
            }
            for (int u = LO_U; u < ca; ++u) {  // long lists
                const Pair ea = zl.pairs[oa + u];
                if (ea.k < klo || ea.k >= khi) continue;
                double *row = Rd + (long long)(ea.k - klo) * K;
                const double va = (double)ea.v;
                for (int w = 0; w < cb; ++w) {
                    const Pair eb = zl.pairs[ob + w];
                    atomicAdd(row + eb.k, va * (double)eb.v);
                }
            }
        }
    }
    __syncthreads();
    const long long row0 = band ? ((long long)cls * LL + di) * K : ((long long)blockIdx.z * gridDim.x + blockIdx.x) * K;
    for (int i = threadIdx.x; i < (khi - klo) * K; i += LO_THREADS) {
        const int k = klo + i / K, k2 = i % K;
        if (!band || k <= k2) out[(row0 + k) * K + k2] = Rd[i];
    }
}

// Rl[lag][a][b] = sum over the chunks z of part[z][delta][a][b] for the lag delta >= 0,
// and Rl[-lag][b][a] = the same sum (R_{-delta} = R_delta^T), through a 32 x 32 LDS
// tile so that both writes are coalesced.  Grid (delta, tiles of a, tiles of b).
constexpr int LS_T = 32;

template <int MM>
__global__ __launch_bounds__(256) void k_lag_sum(int K, int n_chunks, const double *__restrict__ part,
                                                 double *__restrict__ Rl) {
    constexpr int L = 2 * MM - 1, LL = L * L, centre = (LL - 1) / 2, nlag = (LL + 1) / 2;
    __shared__ double t[LS_T][LS_T + 1];
    const int dl = blockIdx.x, a0 = blockIdx.y * LS_T, b0 = blockIdx.z * LS_T;
    for (int i = threadIdx.x; i < LS_T * LS_T; i += 256) {
        const int ia = i / LS_T, ib = i % LS_T, a = a0 + ia, b = b0 + ib;
        if (a >= K || b >= K) continue;
        double v = 0.0;
        for (int z = 0; z < n_chunks; ++z) v += part[(((long long)z * nlag + dl) * K + a) * K + b];
        t[ia][ib] = v;
        Rl[((long long)(centre + dl) * K + a) * K + b] = v;
    }
    if (dl == 0) return;  // R_0 is written once (as summed for (a, b))
    __syncthreads();
    for (int i = threadIdx.x; i < LS_T * LS_T; i += 256) {
        const int ib = i / LS_T, ia = i % LS_T, a = a0 + ia, b = b0 + ib;
        if (a >= K || b >= K) continue;
        Rl[((long long)(centre - dl) * K + b) * K + a] = t[ia][ib];
    }
}

// Filter-major runs for the lags delta = (dy, dx) >= 0 (dy > 0, or dy = 0 and
// dx >= 0).  Workgroup (row range z, chunk of KR first filters k, dy) holds
// S[dx][k][k2] for every dx in LDS.  Each non-zero code a = z_k[y][x] of its
// filters and rows meets the codes of the pixels (y + dy, x + dx), |dx| <= 2c:
// one contiguous run of the per-pixel lists, whose entries carry their columns
// (hence dx).  The codes are visited in groups of G rows, all filters of the
// chunk per group, so that the runs that share a row of partners are read close
// together (L1 reuse).  They are taken LR_NB at a time: first every thread
// resolves one code's run (filter, position, image, run bounds) into an LDS
// descriptor, then LR_SUB lanes read each run at consecutive entries, LR_UNROLL
// loads in flight per lane, and add the products into S.  The workgroups of one
// XCD take neighbouring row ranges, so that their L2 holds the runs they read.
// Output as the pixel-slot pass: part[z][delta][k][k2] with z the row range.
constexpr int LR_THREADS = 1024;
constexpr int LR_SUB = 16;     // lanes per run
constexpr int LR_UNROLL = 6;   // run entries in flight per lane
constexpr int LR_NB = 512;     // descriptors per batch
constexpr int LR_SEG = 256;    // (row group, filter) segments per workgroup
constexpr int LR_LDS = 80 * 1024;
struct RunDesc {
    unsigned j0, len, sidx;
    float va;
};

template <int MM>
__global__ __launch_bounds__(LR_THREADS, 8) void k_lag_rows(const ImgInfo *__restrict__ imgs, int R, int K, int KR,
                                                          int nkc, int P, const unsigned *__restrict__ fm_off,
                                                          const FmCode *__restrict__ fm,
                                                          const unsigned *__restrict__ off,
                                                          const XPair *__restrict__ xp, double *__restrict__ out) {
    constexpr int C2 = 2 * (MM / 2), L = 2 * MM - 1, LL = L * L, nlag = (LL + 1) / 2;
    extern __shared__ double S[];  // [L][KR][K], then the descriptors and the segment table
    RunDesc *desc = reinterpret_cast<RunDesc *>(S + (size_t)L * KR * K);
    unsigned *sst = reinterpret_cast<unsigned *>(desc + LR_NB);  // [LR_SEG] first code of the segment
    unsigned *spr = sst + LR_SEG;                                // [LR_SEG + 1] codes before the segment
    const int per = P / N_XCD;
    const int b = (int)blockIdx.x, xcd = b % N_XCD, bi = b / N_XCD;
    const int z = xcd * per + bi % per, rest = bi / per;
    const int kc = rest % nkc, dy = rest / nkc;
    const int k0 = kc * KR, nk = min(KR, K - k0);
    const int r0 = (int)((long long)R * z / P), r1 = (int)((long long)R * (z + 1) / P);
    const int KRK = KR * K;
    // segments (row group g, filter kk) in the order g major: G rows per group
    const int gmax = LR_SEG / nk;  // groups that fit the table
    const int G = max(8, (r1 - r0 + gmax - 1) / gmax);
    const int ng = (r1 - r0 + G - 1) / G, nseg = ng * nk;
    for (int t = threadIdx.x; t < L * KRK; t += LR_THREADS) S[t] = 0.0;
    for (int sgi = threadIdx.x; sgi <= nseg; sgi += LR_THREADS) {
        // codes before segment (g, kk): all filters' codes of the rows before group g,
        // and the filters before kk in group g
        const int g = sgi / nk, kk = sgi - g * nk;
        const int rg = min(r1, r0 + g * G), re = min(r1, rg + G);
        unsigned before = 0;
        for (int q = 0; q < nk; ++q) {
            const long long fr = (long long)(k0 + q) * R;
            const unsigned base = fm_off[fr + r0];
            before += fm_off[fr + (q < kk ? re : rg)] - base;
        }
        spr[sgi] = before;
        if (sgi < nseg) sst[sgi] = fm_off[(long long)(k0 + kk) * R + rg];
    }
    __syncthreads();
    const unsigned na = spr[nseg];
    const int lane = (int)threadIdx.x % LR_SUB, sg = (int)threadIdx.x / LR_SUB;
    for (unsigned v0 = 0; v0 < na; v0 += LR_NB) {
        if (threadIdx.x < LR_NB) {
            RunDesc dsc{0u, 0u, 0, 0.f};
            const unsigned v = v0 + threadIdx.x;
            if (v < na) {
                int lo = 0, hi = nseg - 1;  // segment of the v-th code: the last one with spr <= v
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (spr[mid] <= v) lo = mid;
                    else hi = mid - 1;
                }
                const int kk = lo % nk;
                const FmCode a = fm[sst[lo] + (v - spr[lo])];
                const ImgInfo im = imgs[a.img];
                const int y2 = (int)(a.yx >> 16) + dy, x = (int)(a.yx & 0xffffu);
                if (y2 < im.H) {
                    const int xlo = max(0, x - (dy > 0 ? C2 : 0)), xhi = min(im.W - 1, x + C2);
                    const long long rb = im.pix_off + (long long)y2 * im.W;
                    dsc.j0 = off[rb + xlo];
                    dsc.len = off[rb + xhi + 1] - dsc.j0;
                    // byte offset of slot (dx = x_b - x, row kk) is sidx + the entry's tag, modulo 2^32
                    dsc.sidx = ((unsigned)kk * (unsigned)K - (unsigned)(x - C2) * (unsigned)KRK) * 8u;
                    dsc.va = a.v;
                }
            }
            desc[threadIdx.x] = dsc;
        }
        __syncthreads();
        for (int di = sg; di < LR_NB; di += LR_THREADS / LR_SUB) {
            const RunDesc dsc = desc[di];
            const double va = (double)dsc.va;
            // the run read from the 64-byte boundary below its first entry; loads past
            // its end repeat the last entry, so that no further cache sector is touched
            const unsigned ja = dsc.j0 & ~7u, skip = dsc.j0 - ja;
            const unsigned span = dsc.len ? dsc.len + skip : 0u;
            const XPair *qa = xp + ja;
            char *Sb = reinterpret_cast<char *>(S);
            for (unsigned t0 = 0; t0 < span; t0 += LR_SUB * LR_UNROLL) {
                XPair e[LR_UNROLL];
#pragma unroll
                for (int u = 0; u < LR_UNROLL; ++u) e[u] = qa[min(t0 + lane + u * LR_SUB, span - 1)];
#pragma unroll
                for (int u = 0; u < LR_UNROLL; ++u) {
                    const unsigned t = t0 + lane + u * LR_SUB;
                    if (t < span && t >= skip)
                        atomicAdd(reinterpret_cast<double *>(Sb + (dsc.sidx + e[u].off)), va * (double)e[u].v);
                }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < L * nk * K; t += LR_THREADS) {
        const int sl = t / (nk * K), rem = t - sl * (nk * K), kk = rem / K, k2 = rem - kk * K;
        const int dx = sl - C2;
        if (dy == 0 && dx < 0) continue;
        out[(((long long)z * nlag + dy * L + dx) * K + k0 + kk) * K + k2] = S[sl * KRK + kk * K + k2];
    }
}

// Product with the zero-padded normal matrix of the batch, whose entry
// (k, s; k2, s2) is the lag sum R_{s - s2}[k][k2] (block Toeplitz in the taps):
// part[chunk][k][s] = sum_{k2 in chunk} sum_{s2} R_{s - s2}[k][k2] v[k2][s2], FP64.
// The vector comes as the previous power-iteration product w and the block
// partial sums of its squared norm: v = w / ||w||, rounded to FP32 as stored.
// Rf is the FP32 copy of the lag sums in [k][k2][lag] order, so that the rows of a
// workgroup's partner chunk are one contiguous range.  Workgroup (k, chunk of
// RM_KB partner filters); thread (k2, tap row s_y) keeps the m outputs of its row
// in registers and reads each lag row once per s2_y; the partner filters are then
// summed in a fixed order.
// Sum of a[0, n) by the 64 lanes of the first wave: lane l adds a[l], a[l + 64], ...
// in order, then a fixed butterfly; every lane ends with the same total.
__device__ __forceinline__ double wave_sum_strided(const double *__restrict__ a, int n) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) t += a[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    return t;
}

constexpr int RM_KB = 16;
constexpr int RM_LB = 48;  // loads in flight per thread (RM_KB LL / threads for m = 11: one round trip)

template <int MM>
__global__ __launch_bounds__(MM *RM_KB) void k_lag_matvec(int K, const float *__restrict__ Rf,
                                                          const float *__restrict__ w,
                                                          const double *__restrict__ nparts, int n_nparts,
                                                          double *__restrict__ part) {
    constexpr int C = MM / 2, M = MM * MM, L = 2 * MM - 1, LL = L * L, NT = MM * RM_KB;
    __shared__ float r[RM_KB * LL];
    __shared__ double vv[RM_KB][M];
    __shared__ double inv_s;
    const int k = blockIdx.x, ch = blockIdx.y;
    const int k2lo = ch * RM_KB, nk = min(RM_KB, K - k2lo);
    if (threadIdx.x < 64) {
        const double nn = wave_sum_strided(nparts, n_nparts);
        if (threadIdx.x == 0) inv_s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    }
    const float *src = Rf + ((long long)k * K + k2lo) * LL;
    const int nr = nk * LL;
    for (int i0 = threadIdx.x; i0 < nr; i0 += NT * RM_LB) {
        float t[RM_LB];
#pragma unroll
        for (int u = 0; u < RM_LB; ++u) {
            const int i = i0 + u * NT;
            t[u] = i < nr ? src[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < RM_LB; ++u) {
            const int i = i0 + u * NT;
            if (i < nr) r[i] = t[u];
        }
    }
    __syncthreads();
    const double inv = inv_s;
    for (int i = threadIdx.x; i < nk * M; i += NT)
        vv[i / M][i % M] = (double)(float)((double)w[(long long)k2lo * M + i] * inv);
    __syncthreads();
    const int j = threadIdx.x / MM, sy = threadIdx.x % MM;
    double acc[MM];
#pragma unroll
    for (int sx = 0; sx < MM; ++sx) acc[sx] = 0.0;
    if (j < nk) {
        for (int s2y = 0; s2y < MM; ++s2y) {
            const float *rrow = &r[j * LL + (sy - s2y + 2 * C) * L];  // lags (dy, dx = sx - s2x + 2c)
            const double *vrow = &vv[j][s2y * MM];
            double rv[L], vx[MM];
#pragma clang loop unroll(full)
            for (int i = 0; i < L; ++i) rv[i] = (double)rrow[i];
#pragma clang loop unroll(full)
            for (int i = 0; i < MM; ++i) vx[i] = vrow[i];
#pragma clang loop unroll(full)
            for (int sx = 0; sx < MM; ++sx)
#pragma clang loop unroll(full)
                for (int s2x = 0; s2x < MM; ++s2x) acc[sx] = fma(rv[sx - s2x + 2 * C], vx[s2x], acc[sx]);
        }
    }
    __syncthreads();
    double *red = &vv[0][0];  // [RM_KB][M], reuses the vector rows
#pragma unroll
    for (int sx = 0; sx < MM; ++sx) red[j * M + sy * MM + sx] = acc[sx];
    __syncthreads();
    for (int s = threadIdx.x; s < M; s += NT) {
        double t = 0.0;
        for (int jj = 0; jj < nk; ++jj) t += red[jj * M + s];
        part[((long long)ch * K + k) * M + s] = t;
    }
}

// Rf[a][b][lag] = (float) Rl[lag][a][b] through 32 x 32 LDS tiles (both sides coalesced).
// Grid (a, tiles of b, tiles of lags).
template <int MM>
__global__ __launch_bounds__(256) void k_lag_to_f32_t(int K, const double *__restrict__ Rl, float *__restrict__ Rf) {
    constexpr int L = 2 * MM - 1, LL = L * L;
    __shared__ float t[32][33];
    const int a = blockIdx.x, b0 = blockIdx.y * 32, l0 = blockIdx.z * 32;
    for (int i = threadIdx.x; i < 32 * 32; i += 256) {
        const int il = i / 32, ib = i % 32, lag = l0 + il, b = b0 + ib;
        if (lag < LL && b < K) t[il][ib] = (float)Rl[((long long)lag * K + a) * K + b];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * 32; i += 256) {
        const int ib = i / 32, il = i % 32, lag = l0 + il, b = b0 + ib;
        if (lag < LL && b < K) Rf[((long long)a * K + b) * LL + lag] = t[il][ib];
    }
}

// One power-iteration reduction: w = sum of the chunk partials (rounded to FP32),
// and per workgroup the partial sums of ||w||^2 and of v . w, with v the vector
// of this product (w_prev / ||w_prev||, as the matvec formed it).
constexpr int PR_THREADS = 256;

__global__ __launch_bounds__(PR_THREADS) void k_power_reduce(const double *__restrict__ part, int nch, int n,
                                                             float *__restrict__ w_out, const float *__restrict__ w_prev,
                                                             const double *__restrict__ nparts_prev, int n_nparts,
                                                             double *__restrict__ nparts_out,
                                                             double *__restrict__ dparts_out) {
    __shared__ double inv_s, rn[PR_THREADS], rd[PR_THREADS];
    if (threadIdx.x < 64) {
        const double nn = wave_sum_strided(nparts_prev, n_nparts);
        if (threadIdx.x == 0) inv_s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    }
    __syncthreads();
    const int i = blockIdx.x * PR_THREADS + threadIdx.x;
    double nn = 0.0, dot = 0.0;
    if (i < n) {
        double sum = 0.0;
        for (int c = 0; c < nch; ++c) sum += part[(long long)c * n + i];
        const float wf = (float)sum;
        w_out[i] = wf;
        const double v = (double)(float)((double)w_prev[i] * inv_s);
        nn = (double)wf * (double)wf;
        dot = v * (double)wf;
    }
    rn[threadIdx.x] = nn;
    rd[threadIdx.x] = dot;
    __syncthreads();
    for (int o = PR_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            rn[threadIdx.x] += rn[threadIdx.x + o];
            rd[threadIdx.x] += rd[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nparts_out[blockIdx.x] = rn[0];
        dparts_out[blockIdx.x] = rd[0];
    }
}

// The starting vector's norm partials: nparts = (nn0, 0, ..., 0).
__global__ void k_power_start(double *nparts, int nb, double nn0) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x) nparts[i] = i == 0 ? nn0 : 0.0;
}

// lam = v . w of the last product (0 when w = 0).
__global__ void k_power_final(const double *__restrict__ nparts, const double *__restrict__ dparts, int nb,
                              double *lam) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double nn = 0.0, dot = 0.0;
    for (int i = 0; i < nb; ++i) {
        nn += nparts[i];
        dot += dparts[i];
    }
    *lam = nn > 0.0 ? dot : 0.0;
}

// C_bar(k, k2) += R - E_top - E_bottom - E_left - E_right for every stored block
// k <= k2 (one workgroup per block, blockIdx.x = its upper-triangle index).
// Each workgroup reads and writes its own block with coalesced accesses.  C_bar is
// streamed with non-temporal loads and stores (each entry is touched once per
// mini-batch), so that it does not evict the lag sums that the power iteration
// beside it reads 20 times.
constexpr int EX_THREADS = 512;
constexpr int EX_BATCH = 16;

template <int MM>
__global__ __launch_bounds__(EX_THREADS) void k_sur_expand(int K, const double *__restrict__ Rl,
                                                           const double *__restrict__ Es,
                                                           const unsigned short *__restrict__ tab,
                                                           double *__restrict__ Cbar, const float *__restrict__ d,
                                                           double *__restrict__ part) {
    constexpr int C = MM / 2, M = MM * MM, M2 = M * M, L = 2 * MM - 1, LL = L * L;
    constexpr int NC = C > 0 ? C : 1;
    // Band prefix sums ec[side][a][b] = sum_{j <= a} E_side,j(delta) over the lags delta at
    // which a band sum can be non-zero: |dy| < c for the top and bottom bands (b = (dy +
    // c - 1) L + dx + 2c), |dx| < c for the left and right ones (b = (dy + 2c)(2c - 1) +
    // dx + c - 1); at every other lag all of them are 0.
    constexpr int NB = (C > 0 ? 2 * C - 1 : 1) * L;
    __shared__ double r[LL];
    __shared__ double ec[4][NC][NB];
    __shared__ double ya[M], yb[M], dka[M], dkb[M];
    // decode the upper-triangle block index into (k, k2); neighbouring blocks
    // (which read neighbouring lag and band sums) share an XCD
    const long long bi = xcd_item(tri_block(K, K, K));
    if (bi < 0) return;
    int k = 0;
    while (tri_block(k + 1, k + 1, K) <= bi) ++k;
    const int k2 = k + (int)(bi - tri_block(k, k, K));
    for (int i = threadIdx.x; i < LL; i += EX_THREADS) r[i] = Rl[((long long)i * K + k) * K + k2];
    // band sums: all loads of the block issued EX_BATCH at a time, then the
    // prefix over the band rows j in LDS
    constexpr int NE = 4 * NC * NB;
    for (int i0 = threadIdx.x; i0 < NE && C > 0; i0 += EX_THREADS * EX_BATCH) {
        double ev[EX_BATCH];
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int i = i0 + u * EX_THREADS;
            ev[u] = 0.0;
            if (i >= NE) continue;
            const int cls = i / NB, b = i % NB;  // cls = side * c + j
            const int sd = cls / NC, j = cls % NC;
            const int dy = sd < 2 ? b / L - (C - 1) : b / (2 * C - 1) - 2 * C;
            const int dx = sd < 2 ? b % L - 2 * C : b % (2 * C - 1) - (C - 1);
            const int di = (dy + 2 * C) * L + dx + 2 * C;
            const int dlt = sd == 0 ? -dy : sd == 1 ? dy : sd == 2 ? -dx : dx;
            // band rows j >= min(c, c + dlt) are never read for this lag, and for dlt > j
            // the partner pixel lies outside every image (the sum is 0); neither was formed
            if (j < min(C, C + dlt) && dlt <= j) ev[u] = Es[(((long long)cls * LL + di) * K + k) * K + k2];
        }
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int i = i0 + u * EX_THREADS;
            if (i < NE) (&ec[0][0][0])[i] = ev[u];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * NB && C > 0; i += EX_THREADS) {
        const int sd = i / NB, b = i % NB;
        double acc = 0.0;
        for (int j = 0; j < NC; ++j) {
            acc += ec[sd][j][b];
            ec[sd][j][b] = acc;
        }
    }
    if (d)  // the product C_bar d of the updated block (first filter iteration), fused
        for (int i = threadIdx.x; i < M; i += EX_THREADS) {
            ya[i] = 0.0;
            yb[i] = 0.0;
            dka[i] = (double)d[(long long)k * M + i];
            dkb[i] = (double)d[(long long)k2 * M + i];
        }
    __syncthreads();
    double *blk = Cbar + bi * M2;
    for (int i0 = threadIdx.x; i0 < M2; i0 += EX_THREADS * EX_BATCH) {
        double val[EX_BATCH], old[EX_BATCH];
        int si[EX_BATCH], s2i[EX_BATCH];
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int i = i0 + u * EX_THREADS;
            val[u] = 0.0;
            si[u] = s2i[u] = 0;
            if (i >= M2) continue;
            const int code = tab[i];
            const int di = code >> 7;
            const int t = code & 127;
            const int dy = di / L - (MM - 1), dx = di % L - (MM - 1);
            const int wx = MM - (dx < 0 ? -dx : dx);
            const int sy = max(-C, dy - C) + t / wx, sx = max(-C, dx - C) + t % wx;
            // R minus the codes whose partner window is cut by the image border:
            // the first -s_y rows (top), last s_y rows (bottom), likewise columns
            double v = r[di];
            const bool by = dy > -C && dy < C, bx = dx > -C && dx < C;  // else the band sums are 0
            const int iy = (dy + C - 1) * L + dx + 2 * C, ix = (dy + 2 * C) * (2 * C - 1) + dx + C - 1;
            if (sy < 0 && by) v -= ec[0][-sy - 1][iy];
            if (sy > 0 && by) v -= ec[1][sy - 1][iy];
            if (sx < 0 && bx) v -= ec[2][-sx - 1][ix];
            if (sx > 0 && bx) v -= ec[3][sx - 1][ix];
            val[u] = v;
            si[u] = (sy + C) * MM + sx + C;
            s2i[u] = (sy - dy + C) * MM + sx - dx + C;
        }
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int i = i0 + u * EX_THREADS;
            old[u] = i < M2 ? __builtin_nontemporal_load(&blk[i]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int i = i0 + u * EX_THREADS;
            if (i >= M2) continue;
            const double nv = old[u] + val[u];
            __builtin_nontemporal_store(nv, &blk[i]);
            if (d) {
                // entry (k, s; k2, s2 = s - delta): row k gets C d_k2, row k2 gets C^T d_k
                atomicAdd(&ya[si[u]], nv * dkb[s2i[u]]);
                if (k != k2) atomicAdd(&yb[s2i[u]], nv * dka[si[u]]);
            }
        }
    }
    if (d) {
        __syncthreads();
        // part layout of the product: [k][k2][2][M]
        double *pp = part + (((long long)k * K + k2) * 2) * M;
        for (int i = threadIdx.x; i < M; i += EX_THREADS) {
            pp[i] = ya[i];
            pp[M + i] = yb[i];
        }
    }
}

// E_corners: the ring pixels p in the four c x c corner blocks outside an image
// were subtracted twice; add back the products of all pairs of codes in their
// windows (at most c x c image pixels each).  One workgroup per (image, corner),
// threads over pairs of window pixels; FP64 atomics into C_bar.
template <int MM>
__global__ __launch_bounds__(256) void k_sur_corner(const ImgInfo *imgs, int K, Lists zl, double *__restrict__ Cbar) {
    constexpr int C = MM / 2, M = MM * MM, M2 = M * M;
    __shared__ int cq[M];  // window pixels inside the image (tap index s = p - q)
    __shared__ long long cg[M];
    __shared__ int ncell;
    const ImgInfo im = imgs[blockIdx.x];
    const int corner = blockIdx.y, ring = blockIdx.z;
    const int i = ring / C + 1, j = ring % C + 1;
    const int py = (corner & 1) ? im.H - 1 + i : -i;
    const int px = (corner & 2) ? im.W - 1 + j : -j;
    if (threadIdx.x == 0) ncell = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < M; t += 256) {
        const int qy = py - (t / MM - C), qx = px - (t % MM - C);  // q = p - s
        if (qy < 0 || qy >= im.H || qx < 0 || qx >= im.W) continue;
        const int slot = atomicAdd(&ncell, 1);
        cq[slot] = t;
        cg[slot] = im.pix_off + (long long)qy * im.W + qx;
    }
    __syncthreads();
    const int n = ncell;
    for (int pi = threadIdx.x; pi < n * n; pi += 256) {
        const int a = pi / n, b = pi % n;
        const int sa = cq[a], sb = cq[b];
        const int say = sa / MM - C, sax = sa % MM - C, sby = sb / MM - C, sbx = sb % MM - C;
        const int dy = say - sby, dx = sax - sbx;
        const int wy = MM - (dy < 0 ? -dy : dy), wx = MM - (dx < 0 ? -dx : dx);
        const int sylo = max(-C, dy - C), sxlo = max(-C, dx - C);
        const long long within = (long long)lagp(dy, MM) * M + wy * lagp(dx, MM) + (say - sylo) * wx + (sax - sxlo);
        const int ca = zl.cnt[cg[a]], cb = zl.cnt[cg[b]];
        const unsigned oa = zl.off[cg[a]], ob = zl.off[cg[b]];
        // entry (k_a, s_a; k_b, s_b) is stored when k_a <= k_b; the mirror of an
        // entry with k_a > k_b comes from the pair (b, a)
        for (int u = 0; u < ca; ++u) {
            const Pair ea = zl.pairs[oa + u];
            for (int w = 0; w < cb; ++w) {
                const Pair eb = zl.pairs[ob + w];
                if (ea.k > eb.k) continue;
                atomicAdd(Cbar + tri_block(ea.k, eb.k, K) * M2 + within, (double)ea.v * (double)eb.v);
            }
        }
    }
}

// ---- y = C_bar d using the symmetric half --------------------------------------
// Block (k, k2 >= k) streams its lag-layout block once: thread t plays tap s = t
// of row k (y_k += C(k,k2) d_k2) and tap s2 = t of row k2 (y_k2 += C(k,k2)^T d_k),
// walking the lags in a fixed order, so the result is deterministic.  Partials
// are reduced per row in a fixed order.
constexpr int MV_THREADS = 128;

template <int MM>
__global__ __launch_bounds__(MV_THREADS) void k_sur_matvec(int K, const double *__restrict__ Cbar,
                                                           const float *__restrict__ d, double *__restrict__ part) {
    constexpr int C = MM / 2, M = MM * MM, M2 = M * M;
    __shared__ double da[M], db[M];
    const int k = blockIdx.y, k2 = blockIdx.x;
    if (k2 < k) return;
    for (int i = threadIdx.x; i < M; i += MV_THREADS) {
        da[i] = (double)d[(long long)k * M + i];
        db[i] = (double)d[(long long)k2 * M + i];
    }
    __syncthreads();
    const double *blk = Cbar + tri_block(k, k2, K) * M2;
    const int t = threadIdx.x;
    const bool active = t < M;
    const int ty = active ? t / MM - C : 0, tx = active ? t % MM - C : 0;
    const bool both = k2 != k;
    double ya = 0.0, yb = 0.0;
    int off = 0;
    for (int dy = -(MM - 1); dy <= MM - 1; ++dy) {
        const int wy = MM - (dy < 0 ? -dy : dy);
        const int sylo = max(-C, dy - C), syhi = min(C, dy + C);
#pragma unroll 3
        for (int dx = -(MM - 1); dx <= MM - 1; ++dx) {
            const int wx = MM - (dx < 0 ? -dx : dx);
            const int sxlo = max(-C, dx - C), sxhi = min(C, dx + C);
            if (active) {
                // row role: s = t, s2 = t - delta
                if (ty >= sylo && ty <= syhi && tx >= sxlo && tx <= sxhi)
                    ya += blk[off + (ty - sylo) * wx + (tx - sxlo)] * db[(ty - dy + C) * MM + (tx - dx + C)];
                // column role: s2 = t, s = t + delta
                const int uy = ty + dy, ux = tx + dx;
                if (both && uy >= sylo && uy <= syhi && ux >= sxlo && ux <= sxhi)
                    yb += blk[off + (uy - sylo) * wx + (ux - sxlo)] * da[(uy + C) * MM + (ux + C)];
            }
            off += wy * wx;
        }
    }
    // part layout: [k][k2][2][M]
    if (active) {
        double *pp = part + (((long long)k * K + k2) * 2) * M;
        pp[t] = ya;
        pp[M + t] = yb;
    }
}

// y[k] = sum_{k2 >= k} part[k][k2][0] + sum_{k1 < k} part[k1][k][1], fixed order.
__global__ void k_sur_matvec_reduce(int K, int M, const double *__restrict__ part, double *__restrict__ y) {
    const int k = blockIdx.x;
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        double s = 0.0;
        for (int k1 = 0; k1 < k; ++k1) s += part[(((long long)k1 * K + k) * 2 + 1) * M + i];
        for (int k2 = k; k2 < K; ++k2) s += part[(((long long)k * K + k2) * 2) * M + i];
        y[(long long)k * M + i] = s;
    }
}

template <int MM>
hipError_t sur_block_impl(const Geometry &g, int K, int R, const unsigned *fm_off, const FmCode *fm,
                          const unsigned char *W, double *C, hipStream_t s) {
    SCSC_LAUNCH(k_sur_block<MM>, dim3(K, K), dim3(SB_THREADS), 0, s, g.d_img, g.n_img, K, R, fm_off, fm, W, C);
    return hipGetLastError();
}

template <int MM>
hipError_t sur_mv_impl(int K, const double *C, const float *d, double *part, double *y, hipStream_t s) {
    SCSC_LAUNCH(k_sur_matvec<MM>, dim3(K, K), dim3(MV_THREADS), 0, s, K, C, d, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_sur_matvec_reduce, dim3(K), dim3(128), 0, s, K, MM * MM, part, y);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fm_lists(const Geometry &g, int K, Lists z, unsigned *fm_cnt, unsigned *fm_off, FmCode *fm,
                           unsigned long long *scan_tmp, unsigned long long *total64, hipStream_t s) {
    const int R = g.n_rows;
    SCSC_LAUNCH(k_fm_count, dim3(R), dim3(256), sizeof(unsigned) * (size_t)K, s, g.d_img, g.d_row_img, z, R,
                K, fm_cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan(fm_cnt, fm_off, (long long)K * R, scan_tmp, total64, s)) != hipSuccess) return e;
    // bitmaps of the widest row when they fit, else the scanning fallback
    const int nww = (g.max_side + 63) / 64;
    const size_t bm_bytes = sizeof(unsigned long long) * (size_t)K * nww;
    const bool use_bm = bm_bytes <= (size_t)FM_BM_BYTES;
    SCSC_LAUNCH(k_fm_fill, dim3(R), dim3(256), use_bm ? bm_bytes : 0, s, g.d_img, g.d_row_img, z, R, K,
                use_bm ? nww : 0, fm_off, fm);
    return hipGetLastError();
}

hipError_t launch_surrogate_blocks(const Geometry &g, int K, int m, const unsigned *fm_off, const FmCode *fm,
                                   const unsigned char *W, double *C, hipStream_t s) {
    const int R = g.n_rows;
    switch (m) {
        case 3: return sur_block_impl<3>(g, K, R, fm_off, fm, W, C, s);
        case 5: return sur_block_impl<5>(g, K, R, fm_off, fm, W, C, s);
        case 7: return sur_block_impl<7>(g, K, R, fm_off, fm, W, C, s);
        case 9: return sur_block_impl<9>(g, K, R, fm_off, fm, W, C, s);
        case 11: return sur_block_impl<11>(g, K, R, fm_off, fm, W, C, s);
        default: return hipErrorInvalidValue;
    }
}

long long surrogate_matvec_partial_elems(int K, int m) { return (long long)K * K * 2 * m * m; }

hipError_t launch_surrogate_matvec(int K, int m, const double *C, const float *d, double *partial, double *y,
                                   hipStream_t s) {
    switch (m) {
        case 3: return sur_mv_impl<3>(K, C, d, partial, y, s);
        case 5: return sur_mv_impl<5>(K, C, d, partial, y, s);
        case 7: return sur_mv_impl<7>(K, C, d, partial, y, s);
        case 9: return sur_mv_impl<9>(K, C, d, partial, y, s);
        case 11: return sur_mv_impl<11>(K, C, d, partial, y, s);
        default: return hipErrorInvalidValue;
    }
}

long long surrogate_lag_elems(int K, int m) { return (long long)K * K * (2 * m - 1) * (2 * m - 1); }

namespace {
struct LagPlan {
    int KC, nkc, nlag;
    long long P;     // pixel chunks of the pixel-slot pass
    int KR, nkr, PR;  // filter-major runs: filters per chunk, chunks, row ranges (0: not usable)
};

template <int MM>
LagPlan lag_plan(const Geometry &g, int K) {
    constexpr int L = 2 * MM - 1, LL = L * L;
    LagPlan pl;
    pl.KC = std::max(1, std::min(K, (80 * 1024) / (8 * K)));
    pl.nkc = (K + pl.KC - 1) / pl.KC;
    pl.nlag = (LL + 1) / 2;
    // pixel chunks: enough workgroups to cover the chip a few times, at least 2048 pixels each
    pl.P = std::max(1LL, std::min(2048LL / ((long long)pl.nlag * pl.nkc), (long long)(g.n_pix / 2048)));
    pl.KR = pl.nkr = pl.PR = 0;
    const long long per_filter = 8LL * L * K, fixed = (long long)sizeof(RunDesc) * LR_NB + 8LL * LR_SEG + 4;
    if (K <= 65535 && g.max_side <= 65535 && g.n_rows > 0 && per_filter + fixed <= LR_LDS) {
        pl.KR = (int)std::min<long long>(K, (LR_LDS - fixed) / per_filter);
        pl.nkr = (K + pl.KR - 1) / pl.KR;
        const long long ny = MM / 2 * 2 + 1;
        // row ranges: a multiple of the XCD count, about 2048 workgroups, ranges of >= 8 rows
        long long q = (2048 + N_XCD * pl.nkr * ny - 1) / (N_XCD * pl.nkr * ny);
        q = std::max(1LL, std::min(q, (long long)g.n_rows / (8 * N_XCD)));
        pl.PR = (int)(N_XCD * q);
    }
    return pl;
}

template <int MM>
unsigned lag_rows_impl(const Geometry &g, int K) {
    const LagPlan pl = lag_plan<MM>(g, K);
    return pl.PR > 0 ? (unsigned)(pl.KR * K) : 0u;
}

template <int MM>
hipError_t sur_lag_impl(const Geometry &g, int K, Lists z, const XPair *xp, const unsigned *fm_off,
                        const FmCode *fm, double *part, double *Rl, double *Es, hipEvent_t sums_done, hipStream_t s) {
    constexpr int Cc = MM / 2, L = 2 * MM - 1, LL = L * L;
    const LagPlan pl = lag_plan<MM>(g, K);
    const size_t shm = sizeof(double) * (size_t)pl.KC * K;
    int nparts = (int)pl.P;
    if (pl.PR > 0 && xp && fm_off && fm) {
        const size_t shr = sizeof(double) * (size_t)L * pl.KR * K + sizeof(RunDesc) * LR_NB +
                           sizeof(unsigned) * (2 * (size_t)LR_SEG + 1);
        const unsigned nb = (unsigned)((long long)pl.PR * pl.nkr * (Cc * 2 + 1));
        SCSC_LAUNCH(k_lag_rows<MM>, dim3(nb), dim3(LR_THREADS), shr, s, g.d_img, g.n_rows, K, pl.KR, pl.nkr,
                    pl.PR, fm_off, fm, z.off, xp, part);
        nparts = pl.PR;
    } else {
        SCSC_LAUNCH(k_lag_outer<MM>, dim3(pl.nlag, pl.nkc, (unsigned)pl.P), dim3(LO_THREADS), shm, s, g.d_img,
                    g.n_img, (long long)g.n_pix, g.max_side, K, z, 0, pl.KC, part);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nt = (unsigned)((K + LS_T - 1) / LS_T);
    SCSC_LAUNCH(k_lag_sum<MM>, dim3(pl.nlag, nt, nt), dim3(256), 0, s, K, nparts, part, Rl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sums_done && (e = hipEventRecord(sums_done, s)) != hipSuccess) return e;
    if (Cc > 0 && Es) {
        SCSC_LAUNCH(k_lag_outer<MM>, dim3(Cc * L, pl.nkc, 4 * Cc), dim3(LO_THREADS), shm, s, g.d_img, g.n_img,
                    (long long)g.n_pix, g.max_side, K, z, 1, pl.KC, Es);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int MM>
long long lag_part_impl(const Geometry &g, int K) {
    const LagPlan pl = lag_plan<MM>(g, K);
    return std::max<long long>(pl.P, pl.PR) * pl.nlag * (long long)K * K;
}

template <int MM>
hipError_t sur_expand_impl(int K, const double *Rl, const double *Es, unsigned short *tab, double *C, const float *d,
                           double *part, double *y, hipStream_t s) {
    constexpr int L = 2 * MM - 1, LL = L * L;
    SCSC_LAUNCH(k_lag_table<MM>, dim3((LL + 63) / 64), dim3(64), 0, s, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SCSC_LAUNCH(k_sur_expand<MM>, dim3(xcd_grid(tri_block(K, K, K))), dim3(EX_THREADS), 0, s, K, Rl, Es, tab,
                C, d, part);
    if (d) {
        if ((e = hipGetLastError()) != hipSuccess) return e;
        SCSC_LAUNCH(k_sur_matvec_reduce, dim3(K), dim3(128), 0, s, K, MM * MM, part, y);
    }
    return hipGetLastError();
}

template <int MM>
hipError_t lag_matvec_impl(int K, const float *Rf, const float *w, const double *nparts, int n_nparts, double *part,
                           hipStream_t s) {
    SCSC_LAUNCH(k_lag_matvec<MM>, dim3(K, (K + RM_KB - 1) / RM_KB), dim3(MM * RM_KB), 0, s, K, Rf, w, nparts,
                n_nparts, part);
    return hipGetLastError();
}

template <int MM>
hipError_t lag_to_f32_impl(int K, const double *Rl, float *Rf, hipStream_t s) {
    constexpr int L = 2 * MM - 1, LL = L * L;
    SCSC_LAUNCH(k_lag_to_f32_t<MM>, dim3(K, (K + 31) / 32, (LL + 31) / 32), dim3(256), 0, s, K, Rl, Rf);
    return hipGetLastError();
}

template <int MM>
hipError_t sur_corner_impl(const Geometry &g, int K, Lists z, double *C, hipStream_t s) {
    constexpr int Cc = MM / 2;
    if (Cc == 0) return hipSuccess;
    SCSC_LAUNCH(k_sur_corner<MM>, dim3(g.n_img, 4, Cc * Cc), dim3(256), 0, s, g.d_img, K, z, C);
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

long long surrogate_lag_part_elems(const Geometry &g, int K, int m) {
    SCSC_DISPATCH_M(m, lag_part_impl, g, K);
}

unsigned lag_rows_stride(const Geometry &g, int K, int m) {
    switch (m) {
        case 3: return lag_rows_impl<3>(g, K);
        case 5: return lag_rows_impl<5>(g, K);
        case 7: return lag_rows_impl<7>(g, K);
        case 9: return lag_rows_impl<9>(g, K);
        case 11: return lag_rows_impl<11>(g, K);
        default: return 0u;
    }
}

hipError_t launch_surrogate_lag(const Geometry &g, int K, int m, Lists z, const XPair *xp, const unsigned *fm_off,
                                const FmCode *fm, double *part, double *Rl, double *Es, hipEvent_t sums_done,
                                hipStream_t s) {
    SCSC_DISPATCH_M(m, sur_lag_impl, g, K, z, xp, fm_off, fm, part, Rl, Es, sums_done, s);
}

hipError_t launch_surrogate_expand(int K, int m, const double *Rl, const double *Es, unsigned short *tab, double *C,
                                   const float *d, double *part, double *y,
                                   hipStream_t s) {
    SCSC_DISPATCH_M(m, sur_expand_impl, K, Rl, Es, tab, C, d, part, y, s);
}

hipError_t launch_surrogate_corner(const Geometry &g, int K, int m, Lists z, double *C, hipStream_t s) {
    SCSC_DISPATCH_M(m, sur_corner_impl, g, K, z, C, s);
}

int lag_matvec_chunks(int K) { return (K + RM_KB - 1) / RM_KB; }

hipError_t launch_lag_matvec(int K, int m, const float *Rf, const float *w, const double *nparts, int n_nparts,
                             double *part, hipStream_t s) {
    SCSC_DISPATCH_M(m, lag_matvec_impl, K, Rf, w, nparts, n_nparts, part, s);
}

hipError_t launch_lag_to_f32(int K, int m, const double *Rl, float *Rf, hipStream_t s) {
    SCSC_DISPATCH_M(m, lag_to_f32_impl, K, Rl, Rf, s);
}

int power_reduce_blocks(int n) { return (n + PR_THREADS - 1) / PR_THREADS; }

hipError_t launch_power_reduce(const double *part, int nch, int n, float *w_out, const float *w_prev,
                               const double *nparts_prev, int n_nparts, double *nparts_out, double *dparts_out,
                               hipStream_t s) {
    SCSC_LAUNCH(k_power_reduce, dim3(power_reduce_blocks(n)), dim3(PR_THREADS), 0, s, part, nch, n, w_out,
                w_prev, nparts_prev, n_nparts, nparts_out, dparts_out);
    return hipGetLastError();
}

hipError_t launch_power_start(double *nparts, int nb, double nn0, hipStream_t s) {
    SCSC_LAUNCH(k_power_start, dim3(1), dim3(256), 0, s, nparts, nb, nn0);
    return hipGetLastError();
}

hipError_t launch_power_final(const double *nparts, const double *dparts, int nb, double *lam, hipStream_t s) {
    SCSC_LAUNCH(k_power_final, dim3(1), dim3(64), 0, s, nparts, dparts, nb, lam);
    return hipGetLastError();
}

}  // namespace scsc
