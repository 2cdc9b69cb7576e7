// C ABI of the gfx950 stochastic-CSC library: handle, workspaces, argument
// validation, batch geometry, and the entry points declared in scsc.h.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "scsc_internal.h"

namespace scsc {
thread_local KernelTiming *kernel_timing = nullptr;
}

using namespace scsc;

namespace {

enum Slot {
    WS_IMG,
    WS_TILES,
    WS_MASK,
    WS_CNT32,
    WS_OFF,
    WS_SCANTMP,
    WS_SCAL,
    WS_PAIRS0,
    WS_PAIRS1,
    WS_NZC0,
    WS_NZC1,
    WS_R,
    WS_PART,
    WS_V,
    WS_W,
    WS_G,
    WS_Y,
    WS_LIP,
    WS_ROWS,
    WS_FMCNT,
    WS_FMOFF,
    WS_FM,
    WS_LAG,
    WS_ES,
    WS_TAB,
    WS_TILESBIG,
    WS_DG,
    WS_GU,
    WS_T,
    WS_XC,
    WS_WC,
    WS_DC,
    WS_LAGF,
    WS_SDA,
    WS_LAGPART,
    WS_PNORM,
    WS_ADA,
    WS_XPAIRS,
    WS_HCNT32,
    WS_HOFF,
    WS_HPAIRS,
    WS_HNZC,
    WS_XE,
    WS_APACK,
    WS_AVEC,
    WS_AZC,
    WS_ADOT,
    WS_ASEG,
    WS_COFF,
    WS_PPART,
    WS_CPART,
    WS_COUNT
};

// Device scalars (doubles / u64) inside WS_SCAL.
enum Scalar {
    SC_TOTAL = 0,
    SC_NNZ = 1,
    SC_LAM = 2,
    SC_LZ = 3,
    SC_OBJ = 4 /* 2 */,
    SC_NNZSUM = 6,
    SC_ETHR = 7 /* two floats: step, threshold */,
    SC_CNNZ = 8 /* non-zero codes after a code step whose statistics are read later */,
    SC_COUNT = 9
};

struct Buffer {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct csc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Buffer ws[WS_COUNT];
    Geometry geo;
    std::vector<int32_t> geo_key;
    bool geo_valid = false;
    double *h_pinned = nullptr;  // host readback staging (SC_COUNT doubles)
    // per-kernel-class event timing (csc_profile_enable / csc_profile_read)
    bool prof = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Rec> recs;
    long long prof_launches[CSC_PK_COUNT] = {};
    double prof_ms[CSC_PK_COUNT] = {};
    // graph replay (csc_set_graph) of the proximal-gradient iterations (slot 0) and of
    // the power iteration on the lag sums (slot 1)
    bool graphs = false;
    bool capturing = false;
    std::vector<uintptr_t> graph_key[2];
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    hipStream_t graph_stream = nullptr;  // capture / replay stream when the handle's stream is the null stream
    // second stream (default priority) for the parts of the online filter step that
    // do not depend on each other, ordered against the handle's stream with events
    hipStream_t side = nullptr;
    hipEvent_t side_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool side_failed = false;
    // a third stream for the third part of a split BF16 code step, with its join event
    hipStream_t side2 = nullptr;
    hipEvent_t side2_ev = nullptr;
    hipEvent_t graph_ev[2] = {nullptr, nullptr};
    // autotuner: launch variant per (kernel, m, K, log2 pixel count, mode)
    bool autotune = true;
    int force_variant = -1;
    std::map<std::array<int, 5>, int> tuned;
    // the split code step's variants: the two best of a screening and the unsplit
    // loop, confirmed on the next three calls (their iteration loops timed with split_ev)
    struct SplitTune {
        int cand[3] = {-1, -1, -1};      // the two best split pairs, and the loop on one stream
        float ms[3] = {-1.f, -1.f, -1.f};  // each candidate's timed call
        int runs = 0;                    // confirmation calls made (one per candidate)
        int pending = -1;                // candidate whose call's events have not been read yet
    };
    std::map<std::array<int, 5>, SplitTune> split_tune;
    hipEvent_t split_ev[2] = {nullptr, nullptr};
    // this device's copy of the fixed scratch array (csc_objective_noalloc), or null if
    // its address could not be obtained when the handle was created
    unsigned char *scratch = nullptr;
    // cap on the handle's device workspaces in bytes (0: none), from SCSC_WORKSPACE_LIMIT at creation
    size_t ws_limit = 0;
    size_t ws_total = 0;
};

namespace {

int fail(csc_ctx *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

hipEvent_t take_event(csc_ctx *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        hipGetLastError();
        return nullptr;
    }
    return e;
}

// Fold finished records into the per-class totals (waits for the events).
void fold_records(csc_ctx *h) {
    for (auto &r : h->recs) {
        float ms = 0.f;
        hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            h->prof_launches[r.cls] += 1;
            h->prof_ms[r.cls] += ms;
        } else {
            hipGetLastError();
        }
        h->ev_pool.push_back(r.a);
        h->ev_pool.push_back(r.b);
    }
    h->recs.clear();
}

// Times the launches of its scope when profiling is on: from the first kernel's start to
// the last kernel's end, with events that the kernels record themselves (SCSC_LAUNCH).
// A scope that launches no kernel of this library (a graph replay) is timed with an
// event pair recorded on the handle's stream around it instead.
struct ProfScope {
    csc_ctx *h;
    int cls;
    hipEvent_t a = nullptr;  // marker-pair timing only
    KernelTiming kt;
    KernelTiming *outer = nullptr;
    bool hooked = false;
    ProfScope(csc_ctx *h_, int cls_, bool markers = false) : h(h_), cls(cls_) {
        if (!h->prof || h->capturing) return;
        if (markers) {
            a = take_event(h);
            if (a) hipEventRecord(a, h->stream);
            return;
        }
        kt.start = take_event(h);
        kt.stop = take_event(h);
        if (kt.start && kt.stop) {
            outer = kernel_timing;
            kernel_timing = &kt;
            hooked = true;
        } else {
            if (kt.start) h->ev_pool.push_back(kt.start);
            if (kt.stop) h->ev_pool.push_back(kt.stop);
        }
    }
    ~ProfScope() {
        if (hooked) {
            kernel_timing = outer;
            if (kt.used) {
                h->recs.push_back(csc_ctx::Rec{cls, kt.start, kt.stop});
            } else {
                h->ev_pool.push_back(kt.start);
                h->ev_pool.push_back(kt.stop);
            }
        } else if (a) {
            hipEvent_t b = take_event(h);
            if (!b) return;
            hipEventRecord(b, h->stream);
            h->recs.push_back(csc_ctx::Rec{cls, a, b});
        }
        if (h->recs.size() > 100000) fold_records(h);
    }
};

#define PROF(cls) ProfScope prof_scope_(h, cls)
#define PROF_MARKERS(cls) ProfScope prof_scope_(h, cls, true)

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(h, CSC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Kernels with several launch variants that compute bit-identical results.
enum TunedKernel { TK_SYNTH = 0, TK_SYNTH_BF16 = 1, TK_SPLIT_BF16 = 2, TK_SPLIT_FP32 = 3 };
constexpr int SYNTH_FP32_VARIANTS = 4;

int ilog2(long long v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

// Launch the variant chosen for `key`.  The first time a key is seen (and the
// stream is not being captured) every variant is timed on the call's own data
// with HIP events and the fastest is kept for the handle's lifetime.  Variants
// write the same outputs from the same inputs, so the extra launches leave the
// call's result unchanged.
hipError_t tuned_launch(csc_ctx *h, const std::array<int, 5> &key, int n_variants,
                        const std::function<hipError_t(int)> &launch, bool representative = true) {
    if (h->force_variant >= 0) return launch(h->force_variant < n_variants ? h->force_variant : 0);
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) return launch(it->second);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!representative || !h->autotune || n_variants < 2 || hipStreamIsCapturing(h->stream, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone) {
        hipGetLastError();
        return launch(0);
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        (void)hipGetLastError();
        if (a) hipEventDestroy(a);
        return launch(0);
    }
    // each variant: one warm-up launch, then the fastest of three timed launches
    int best = 0;
    float best_ms = 0.f;
    hipError_t e = hipSuccess;
    for (int v = 0; v < n_variants && e == hipSuccess; ++v) {
        e = launch(v);
        float vmin = 0.f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            hipEventRecord(a, h->stream);
            e = launch(v);
            hipEventRecord(b, h->stream);
            if (e != hipSuccess) break;
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            if (rep == 0 || ms < vmin) vmin = ms;
        }
        if (e != hipSuccess) break;
        if (std::getenv("SCSC_TUNE_LOG"))
            std::fprintf(stderr, "[scsc tune] kernel %d m %d K %d log2px %d mode %d: variant %d %.1f us\n", key[0],
                         key[1], key[2], key[3], key[4], v, 1e3 * vmin);
        if (v == 0 || vmin < best_ms) {
            best = v;
            best_ms = vmin;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (e != hipSuccess) return e;
    h->tuned[key] = best;
    return hipSuccess;
}

// True when the variant of `key` is fixed (tuned, forced or tuning off), i.e.
// a launch would not time variants.
bool variant_settled(csc_ctx *h, const std::array<int, 5> &key) {
    return h->force_variant >= 0 || !h->autotune || h->tuned.count(key) > 0;
}

// Variant chosen for `key` (-1 when not tuned yet); does not insert.
int tuned_variant(csc_ctx *h, const std::array<int, 5> &key) {
    auto it = h->tuned.find(key);
    return it == h->tuned.end() ? -1 : it->second;
}

std::array<int, 5> synth_key(csc_ctx *h, int K, int m, SynthMode mode, int precision = CSC_FP32) {
    return {precision == CSC_BF16 ? TK_SYNTH_BF16 : TK_SYNTH, m, K, ilog2(h->geo.n_pix), (int)mode};
}

// Synthesis / residual through the tuned launcher (tile shape and threads per
// output pixel).  `representative` marks calls whose code density is typical of
// the key (not the first iterations of a code step from zero codes); only those
// may tune.
void *ws(csc_ctx *h, Slot s, size_t bytes, int *status);

// With BF16 the filters enter as the matrix-core operand: `dA` when the caller
// prepared it (launch_synth_mfma_prep), else prepared here into WS_SDA.
hipError_t synth(csc_ctx *h, int K, int m, Lists L, const float *d, const float *x, const unsigned char *W,
                 float *out, SynthMode mode, bool representative = true, int precision = CSC_FP32,
                 const __bf16 *dA = nullptr) {
    const Geometry &g = h->geo;
    if (precision == CSC_BF16) {
        if (!dA) {
            int st = CSC_OK;
            __bf16 *buf = static_cast<__bf16 *>(ws(h, WS_SDA, sizeof(__bf16) * synth_mfma_prep_elems(K), &st));
            if (!buf) return hipErrorOutOfMemory;
            const hipError_t e = launch_synth_mfma_prep(d, K, m, buf, h->stream);
            if (e != hipSuccess) return e;
            dA = buf;
        }
        return tuned_launch(
            h, synth_key(h, K, m, mode, precision), SYNTH_MFMA_VARIANTS,
            [&](int v) { return launch_synth_mfma(g, K, m, L, dA, x, W, out, (int)mode, v, h->stream); },
            representative);
    }
    return tuned_launch(
        h, synth_key(h, K, m, mode), SYNTH_FP32_VARIANTS,
        [&](int v) { return launch_synth(g, K, m, L, d, x, W, out, mode, v, h->stream); }, representative);
}

// Capture `body` (kernel launches only) into graph slot `slot` the first time `key`
// is seen, then replay it on the handle's stream.  The null stream cannot be
// captured: a private (default-priority) stream is used instead, ordered after
// and before the handle's stream with events.
int graph_replay(csc_ctx *h, int slot, const std::vector<uintptr_t> &key, const std::function<int()> &body) {
    hipStream_t gs = h->stream;
    if (gs == nullptr) {
        if (!h->graph_stream) {
            HIPCHK(hipStreamCreateWithFlags(&h->graph_stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&h->graph_ev[0], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->graph_ev[1], hipEventDisableTiming));
        }
        gs = h->graph_stream;
    }
    hipGraphExec_t &ge = h->graph_exec[slot];
    if (!ge || key != h->graph_key[slot]) {
        if (ge) {
            HIPCHK(hipStreamSynchronize(gs));
            hipGraphExecDestroy(ge);
            ge = nullptr;
        }
        hipStream_t saved = h->stream;
        HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        h->stream = gs;
        h->capturing = true;
        const int cst = body();
        h->capturing = false;
        h->stream = saved;
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(gs, &graph);
        if (cst) {
            if (graph) hipGraphDestroy(graph);
            return cst;
        }
        HIPCHK(ce);
        const hipError_t ie = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        HIPCHK(ie);
        h->graph_key[slot] = key;
    }
    PROF_MARKERS(CSC_PK_GRAPH);
    if (gs != h->stream) {
        HIPCHK(hipEventRecord(h->graph_ev[0], h->stream));
        HIPCHK(hipStreamWaitEvent(gs, h->graph_ev[0], 0));
        HIPCHK(hipGraphLaunch(ge, gs));
        HIPCHK(hipEventRecord(h->graph_ev[1], gs));
        HIPCHK(hipStreamWaitEvent(h->stream, h->graph_ev[1], 0));
    } else {
        HIPCHK(hipGraphLaunch(ge, gs));
    }
    return CSC_OK;
}

// Device workspace of at least `bytes` (contents undefined).  Growing frees the
// old buffer after the stream has drained.
void *ws(csc_ctx *h, Slot s, size_t bytes, int *status) {
    Buffer &b = h->ws[s];
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return b.p;
    size_t want = bytes + bytes / 8;
    if (h->ws_limit && h->ws_total - b.bytes + want > h->ws_limit) {
        *status = fail(h, CSC_ENOMEM, "device workspace of " + std::to_string(want) + " bytes would exceed the " +
                                          "handle's limit of " + std::to_string(h->ws_limit) + " bytes");
        return nullptr;
    }
    if (b.p) {
        hipStreamSynchronize(h->stream);
        hipFree(b.p);
        h->ws_total -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.p, want) != hipSuccess) {
        hipGetLastError();
        b.p = nullptr;
        *status = fail(h, CSC_ENOMEM, "device workspace allocation of " + std::to_string(want) + " bytes failed");
        return nullptr;
    }
    b.bytes = want;
    h->ws_total += want;
    return b.p;
}

#define WS(ptr, type, slot, count)                                                    \
    type *ptr = nullptr;                                                              \
    do {                                                                              \
        int st_ = CSC_OK;                                                             \
        ptr = static_cast<type *>(ws(h, slot, sizeof(type) * (size_t)(count), &st_)); \
        if (!ptr) return st_;                                                         \
    } while (0)

bool supported_m(int m) { return m == 3 || m == 5 || m == 7 || m == 9 || m == 11; }

// Float, int and u16 arrays must be 4-byte aligned, double arrays 8-byte aligned
// (null pointers are checked separately).
int check_aligned(csc_ctx *h, std::initializer_list<const void *> p4, std::initializer_list<const void *> p8 = {}) {
    for (const void *p : p4)
        if (p && reinterpret_cast<uintptr_t>(p) % 4u)
            return fail(h, CSC_EINVAL, "array arguments of 4-byte elements must be 4-byte aligned");
    for (const void *p : p8)
        if (p && reinterpret_cast<uintptr_t>(p) % 8u)
            return fail(h, CSC_EINVAL, "surrogate arrays must be 8-byte aligned");
    return CSC_OK;
}

int check_filters(csc_ctx *h, int K, int m) {
    if (K < 1 || K > MAX_K) return fail(h, CSC_EINVAL, "K must lie in [1, 1024]");
    if (m < 1 || (m & 1) == 0) return fail(h, CSC_EINVAL, "filter side m must be odd and positive");
    if (!supported_m(m)) return fail(h, CSC_EUNSUPPORTED, "filter side m must be one of 3, 5, 7, 9, 11");
    return CSC_OK;
}

int check_images(csc_ctx *h, const csc_images *im) {
    if (!im || !im->hw || im->n < 1) return fail(h, CSC_EINVAL, "images: need n >= 1 and a host hw array");
    if (im->index_base < 0) return fail(h, CSC_EINVAL, "images: index_base must be >= 0");
    long long pix = 0;
    for (int i = 0; i < im->n; ++i) {
        const long long H = im->hw[2 * i], W = im->hw[2 * i + 1];
        if (H < 1 || W < 1) return fail(h, CSC_EINVAL, "images: every H and W must be >= 1");
        pix += H * W;
    }
    if (pix >= (1LL << 31)) return fail(h, CSC_EUNSUPPORTED, "images: total pixel count must be < 2^31");
    return CSC_OK;
}

int check_precision(csc_ctx *h, int precision) {
    if (precision != CSC_FP32 && precision != CSC_BF16) return fail(h, CSC_EINVAL, "unknown precision");
    return CSC_OK;
}

// Image records (packed offsets, tile counts, sampler index, first global row) and
// the TS x TS tile records of a batch, in packing order.
void batch_records(const csc_images *im, std::vector<ImgInfo> &imgs, std::vector<TileInfo> &tiles) {
    imgs.assign(im->n, ImgInfo{});
    tiles.clear();
    long long pix = 0;
    int ntiles = 0, rows = 0;
    for (int i = 0; i < im->n; ++i) {
        ImgInfo &ii = imgs[i];
        ii.H = im->hw[2 * i];
        ii.W = im->hw[2 * i + 1];
        ii.pix_off = pix;
        ii.tiles_y = (ii.H + TS - 1) / TS;
        ii.tiles_x = (ii.W + TS - 1) / TS;
        ii.tile_off = ntiles;
        ii.index = im->index_base + i;
        ii.row_off = rows;
        rows += ii.H;
        for (int ty = 0; ty < ii.tiles_y; ++ty)
            for (int tx = 0; tx < ii.tiles_x; ++tx) tiles.push_back(TileInfo{i, ty, tx, 0});
        ntiles += ii.tiles_y * ii.tiles_x;
        pix += (long long)ii.H * ii.W;
    }
}

// Upload (or reuse) the geometry of a batch.
int geometry(csc_ctx *h, const csc_images *im) {
    std::vector<int32_t> key(im->hw, im->hw + 2 * im->n);
    key.push_back(im->index_base);
    if (h->geo_valid && key == h->geo_key) return CSC_OK;
    Geometry &g = h->geo;
    batch_records(im, g.h_img, g.h_tiles);
    g.h_tiles_big.clear();
    int max_side = 0, rows = 0;
    std::vector<int> row_img;
    for (int i = 0; i < im->n; ++i) {
        const ImgInfo &ii = g.h_img[i];
        rows += ii.H;
        row_img.insert(row_img.end(), ii.H, i);
        for (int ty = 0; ty < (ii.H + TS_BIG - 1) / TS_BIG; ++ty)
            for (int tx = 0; tx < (ii.W + TS_BIG - 1) / TS_BIG; ++tx) g.h_tiles_big.push_back(TileInfo{i, ty, tx, 0});
        max_side = std::max(max_side, std::max(ii.H, ii.W));
    }
    g.n_img = im->n;
    g.n_tiles = (int)g.h_tiles.size();
    g.n_pix = im->n ? g.h_img.back().pix_off + (long long)g.h_img.back().H * g.h_img.back().W : 0;
    g.max_side = max_side;
    g.n_rows = rows;
    g.n_tiles_big = (int)g.h_tiles_big.size();
    h->geo_valid = false;
    WS(dimg, ImgInfo, WS_IMG, g.n_img);
    WS(dtiles, TileInfo, WS_TILES, g.n_tiles);
    WS(drows, int, WS_ROWS, g.n_rows);
    WS(dtb, TileInfo, WS_TILESBIG, g.n_tiles_big);
    HIPCHK(hipMemcpyAsync(dtb, g.h_tiles_big.data(), sizeof(TileInfo) * g.n_tiles_big, hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipMemcpyAsync(drows, row_img.data(), sizeof(int) * g.n_rows, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(dimg, g.h_img.data(), sizeof(ImgInfo) * g.n_img, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(dtiles, g.h_tiles.data(), sizeof(TileInfo) * g.n_tiles, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    g.d_img = dimg;
    g.d_tiles = dtiles;
    g.d_row_img = drows;
    g.d_tiles_big = dtb;
    h->geo_key = key;
    h->geo_valid = true;
    return CSC_OK;
}

int read_scalars(csc_ctx *h, const void *dev, int count) {
    HIPCHK(hipMemcpyAsync(h->h_pinned, dev, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return CSC_OK;
}

int dft_size(int max_side, int m) {
    int P = 1;
    while (P < max_side + m - 1) P *= 2;
    return P;
}

int lipschitz(csc_ctx *h, const float *d, int K, int m, int max_side, double *out) {
    const int P = dft_size(max_side, m);
    WS(tmp, double, WS_LIP, lipschitz_tmp_elems(K, m, P));
    WS(sc, double, WS_SCAL, SC_COUNT);
    {
        PROF(CSC_PK_LIPSCHITZ);
        HIPCHK(launch_lipschitz_code(d, K, m, P, tmp, sc + SC_LZ, h->stream));
    }
    int st = read_scalars(h, sc, SC_COUNT);
    if (st) return st;
    *out = h->h_pinned[SC_LZ];
    return CSC_OK;
}

// Lists of the non-zero codes of a dense z, each pixel's list exactly as long as
// its count (offsets = prefix of the counts).  *nnz_out is the size of the pair
// buffer (an upper bound of the total), for sizing per-entry buffers.  With
// xp_out, the entries are also written tagged for row stride xmul (XPair).
constexpr unsigned long long LIST_BOUND_BYTES = 1ULL << 30;
int build_nonzero_lists(csc_ctx *h, int K, const float *z, Lists *out, unsigned long long *nnz_out = nullptr,
                        const XPair **xp_out = nullptr, unsigned xmul = 0) {
    const Geometry &g = h->geo;
    WS(cnt32, unsigned, WS_CNT32, g.n_pix);
    WS(off, unsigned, WS_OFF, g.n_pix + 1);
    WS(tmp, unsigned long long, WS_SCANTMP, scan_tmp_elems(g.n_pix));
    WS(sc, double, WS_SCAL, SC_COUNT);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(sc + SC_TOTAL);
    {
        PROF(CSC_PK_LISTS);
        HIPCHK(launch_count_nonzero(g, K, z, cnt32, h->stream));
        HIPCHK(launch_scan(cnt32, off, g.n_pix, tmp, total, h->stream));
    }
    // capacity: every coordinate when that bound is modest (no read-back of the
    // count, so the host does not wait for the GPU here), else the exact count
    const unsigned long long bound = (unsigned long long)K * (unsigned long long)g.n_pix;
    unsigned long long nz = bound;
    if (bound >= (1ULL << 32) || bound * (sizeof(Pair) + sizeof(FmCode)) > LIST_BOUND_BYTES) {
        int st = read_scalars(h, sc, SC_COUNT);
        if (st) return st;
        std::memcpy(&nz, &h->h_pinned[SC_TOTAL], sizeof(nz));
        if (nz >= (1ULL << 32)) return fail(h, CSC_EUNSUPPORTED, "more than 2^32 non-zero codes");
    }
    WS(pairs, Pair, WS_PAIRS0, nz + 1);
    WS(nzc, unsigned short, WS_NZC0, g.n_pix);
    XPair *xp = nullptr;
    if (xp_out) {
        WS(xpb, XPair, WS_XPAIRS, nz + 1);
        xp = xpb;
        *xp_out = xp;
    }
    {
        PROF(CSC_PK_LISTS);
        HIPCHK(launch_fill_nonzero(g, K, z, off, pairs, nzc, xp, xmul, h->stream));
    }
    *out = Lists{off, nzc, pairs};
    if (nnz_out) *nnz_out = nz;
    return CSC_OK;
}

// Per-filter lists of the non-zero codes (FmLists), built from exact-capacity pixel lists.
struct FmLists {
    const unsigned *off;
    const FmCode *codes;
};

int build_fm_lists(csc_ctx *h, int K, Lists L, unsigned long long nz, FmLists *out) {
    const Geometry &g = h->geo;
    if (g.max_side > 65535) return fail(h, CSC_EUNSUPPORTED, "filter step: image sides must be < 65536");
    const long long KR = (long long)K * g.n_rows;
    WS(fmcnt, unsigned, WS_FMCNT, KR);
    WS(fmoff, unsigned, WS_FMOFF, KR + 1);
    WS(tmp, unsigned long long, WS_SCANTMP, scan_tmp_elems(KR));
    WS(fm, FmCode, WS_FM, nz + 1);
    WS(sc, double, WS_SCAL, SC_COUNT);
    PROF(CSC_PK_LISTS);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(sc + SC_NNZ);
    HIPCHK(launch_fm_lists(g, K, L, fmcnt, fmoff, fm, tmp, total, h->stream));
    *out = FmLists{fmoff, fm};
    return CSC_OK;
}

// G = sum_i Z_i^T r_i into `G` (FP32, [K][M]) from per-filter lists (FP64 accumulation).
int filter_corr_lists(csc_ctx *h, int K, int m, FmLists F, const float *r, float *G) {
    const Geometry &g = h->geo;
    const int M = m * m;
    const int nch = corr_chunks(K);
    WS(part, double, WS_PART, (size_t)nch * K * M);
    PROF(CSC_PK_CORR);
    HIPCHK(launch_corr_fm(g, K, m, F.off, F.codes, r, nullptr, false, part, h->stream));
    HIPCHK(launch_reduce_partials_f64_to_f32(part, nch, K * M, G, h->stream));
    return CSC_OK;
}

// G = sum_i Z_i^T r_i with BF16 operands on the matrix cores (per-pixel lists).
int filter_corr_bf16(csc_ctx *h, int K, int m, Lists L, const float *r, float *G) {
    const Geometry &g = h->geo;
    WS(part, float, WS_PART, (size_t)corr_mfma_blocks(g, K) * K * m * m);
    PROF(CSC_PK_CORR);
    HIPCHK(launch_corr_mfma(g, K, m, L, r, part, G, h->stream));
    return CSC_OK;
}

// Power iteration on sum_i Z_i^T W_i Z_i; leaves the estimate in the device scalar SC_LAM.
int power_iteration(csc_ctx *h, int K, int m, Lists L, FmLists F, const unsigned char *W, int n_power,
                    int precision) {
    const Geometry &g = h->geo;
    const int M = m * m;
    WS(v, float, WS_V, K * M);
    WS(w, float, WS_W, K * M);
    WS(R, float, WS_R, g.n_pix);
    WS(sc, double, WS_SCAL, SC_COUNT);
    HIPCHK(launch_fill(v, K * M, (float)(1.0 / std::sqrt((double)K * M)), h->stream));
    HIPCHK(hipMemsetAsync(sc + SC_LAM, 0, sizeof(double), h->stream));
    for (int it = 0; it < n_power; ++it) {
        {
            PROF(CSC_PK_SYNTH);
            HIPCHK(synth(h, K, m, L, v, nullptr, W, R, SYNTH_WEIGHTED, true, precision));
        }
        int st = precision == CSC_BF16 ? filter_corr_bf16(h, K, m, L, R, w) : filter_corr_lists(h, K, m, F, R, w);
        if (st) return st;
        PROF(CSC_PK_UPDATE);
        HIPCHK(launch_power_update(v, w, K * M, sc + SC_LAM, h->stream));
    }
    return CSC_OK;
}

// Power iteration on the zero-padded normal matrix given by the lag sums Rl
// (no observation mask); leaves the estimate in the device scalar SC_LAM.
// Power iteration on the lag sums, launched on stream `s` (the handle's stream or
// its side stream); its workspaces are its own, so it may run beside the surrogate
// kernels.
int power_iteration_lag(csc_ctx *h, int K, int m, const double *Rl, int n_power, hipStream_t s) {
    const int M = m * m, n = K * M;
    const int nch = lag_matvec_chunks(K), nb = power_reduce_blocks(n);
    WS(wa, float, WS_V, n);
    WS(wb, float, WS_W, n);
    WS(part, double, WS_PPART, (size_t)nch * n);
    WS(np, double, WS_PNORM, 3 * (size_t)nb);
    WS(sc, double, WS_SCAL, SC_COUNT);
    WS(Rf, float, WS_LAGF, surrogate_lag_elems(K, m));
    HIPCHK(launch_lag_to_f32(K, m, Rl, Rf, s));
    // start: v = the normalised ones vector, given as w = 1 with ||w||^2 = n
    double *na = np, *nbp = np + nb, *dp = np + 2 * nb;
    HIPCHK(launch_fill(wa, n, 1.0f, s));
    HIPCHK(launch_power_start(na, nb, (double)n, s));
    HIPCHK(hipMemsetAsync(sc + SC_LAM, 0, sizeof(double), s));
    // the products only launch kernels (their vectors and norms live on the device),
    // so the same launches can be replayed as a graph; on the handle's stream they
    // take h->stream at launch time, which is the capture stream while a graph is
    // being recorded
    const bool own = s == h->stream;
    auto products = [&]() -> int {
        const hipStream_t ls = own ? h->stream : s;
        float *a = wa, *b = wb;
        double *p = na, *q = nbp;
        for (int it = 0; it < n_power; ++it) {
            PROF(CSC_PK_POWER);
            HIPCHK(launch_lag_matvec(K, m, Rf, a, p, nb, part, ls));
            HIPCHK(launch_power_reduce(part, nch, n, b, a, p, nb, q, dp, ls));
            std::swap(a, b);
            std::swap(p, q);
        }
        if (n_power > 0) HIPCHK(launch_power_final(p, dp, nb, sc + SC_LAM, ls));
        return CSC_OK;
    };
    if (h->graphs && n_power > 0 && own) {
        const std::vector<uintptr_t> key = {(uintptr_t)K, (uintptr_t)m, (uintptr_t)n_power, (uintptr_t)Rf,
                                            (uintptr_t)wa, (uintptr_t)wb, (uintptr_t)part, (uintptr_t)np,
                                            (uintptr_t)sc};
        return graph_replay(h, 1, key, products);
    }
    return products();
}

}  // namespace

// ===========================================================================
// Fixed device scratch of the allocation-free entry point.  Each GPU holds its
// own copy of the array until the process ends.  Host code never passes the
// array's name to a kernel or copy: it uses the per-device address taken once
// with that device current.
// ===========================================================================

static __device__ __align__(256) unsigned char scratch[CSC_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;  // device -> its copy of `scratch`

// With `device` current: the device address of that device's copy of `scratch`.
int scratch_address(int device, unsigned char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hipGetLastError();
            return CSC_EHIP;
        }
        it = g_scratch_addr.emplace(device, static_cast<unsigned char *>(p)).first;
    }
    *out = it->second;
    return CSC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// ===========================================================================
// Entry points
// ===========================================================================

extern "C" int csc_version(void) { return CSC_VERSION; }

extern "C" int csc_create(csc_handle *out, int device, void *stream) {
    if (!out) return CSC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        hipGetLastError();
        return CSC_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) return CSC_EHIP;
    csc_ctx *h = new csc_ctx();
    h->device = device;
    h->stream = static_cast<hipStream_t>(stream);
    if (hipHostMalloc(reinterpret_cast<void **>(&h->h_pinned), sizeof(double) * SC_COUNT, hipHostMallocDefault) !=
        hipSuccess) {
        delete h;
        return CSC_ENOMEM;
    }
    if (scratch_address(device, &h->scratch) != CSC_OK) h->scratch = nullptr;  // reported by csc_objective_noalloc
    if (const char *lim = std::getenv("SCSC_WORKSPACE_LIMIT")) h->ws_limit = std::strtoull(lim, nullptr, 10);
    *out = h;
    return CSC_OK;
}

extern "C" int csc_destroy(csc_handle h) {
    if (!h) return CSC_EINVAL;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    fold_records(h);
    for (auto &ge : h->graph_exec)
        if (ge) hipGraphExecDestroy(ge);
    if (h->graph_stream) {
        hipStreamSynchronize(h->graph_stream);
        hipStreamDestroy(h->graph_stream);
    }
    if (h->side) {
        hipStreamSynchronize(h->side);
        hipStreamDestroy(h->side);
    }
    if (h->side2) {
        hipStreamSynchronize(h->side2);
        hipStreamDestroy(h->side2);
    }
    if (h->side2_ev) hipEventDestroy(h->side2_ev);
    for (auto e : h->side_ev)
        if (e) hipEventDestroy(e);
    for (auto e : h->split_ev)
        if (e) hipEventDestroy(e);
    for (auto e : h->graph_ev)
        if (e) hipEventDestroy(e);
    for (auto e : h->ev_pool) hipEventDestroy(e);
    for (auto &b : h->ws)
        if (b.p) hipFree(b.p);
    if (h->h_pinned) hipHostFree(h->h_pinned);
    delete h;
    return CSC_OK;
}

extern "C" int csc_set_stream(csc_handle h, void *stream) {
    if (!h) return CSC_EINVAL;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    h->stream = static_cast<hipStream_t>(stream);
    return CSC_OK;
}

extern "C" const char *csc_last_error(csc_handle h) { return h ? h->err.c_str() : "null handle"; }

extern "C" int csc_lipschitz_code(csc_handle h, const float *d, int K, int m, int max_side, double *L_out) {
    if (!h) return CSC_EINVAL;
    int st = check_filters(h, K, m);
    if (st) return st;
    if (!d || !L_out) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {d}))) return st;
    if (max_side < 1 || max_side > (1 << 16)) return fail(h, CSC_EINVAL, "max_side must lie in [1, 65536]");
    HIPCHK(hipSetDevice(h->device));
    return lipschitz(h, d, K, m, max_side, L_out);
}

extern "C" int csc_mask(csc_handle h, const csc_images *im, int K, double p, uint64_t seed, uint32_t draw,
                        uint8_t *mask) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, 3);
    if (st) return st;
    if (!(p > 0.0 && p <= 1.0)) return fail(h, CSC_EINVAL, "p must lie in (0, 1]");
    if (!mask) return fail(h, CSC_EINVAL, "null pointer argument");
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;
    const int W32 = (K + 31) / 32;
    WS(mw, unsigned, WS_MASK, (size_t)W32 * g.n_pix);
    WS(cnt32, unsigned, WS_CNT32, g.n_pix);
    const unsigned long long thr = (unsigned long long)std::floor(std::ldexp(p, 32));
    HIPCHK(launch_mask_count(g, K, thr, seed, draw, mw, cnt32, h->stream));
    HIPCHK(launch_expand_mask(g, K, mw, mask, h->stream));
    return CSC_OK;
}

// What a code step hands to a filter step that follows it in the same call
// (csc_online_step): the codes start from zero (z is not read and, when null,
// not written), and the statistics are left on the device (SC_CNNZ, SC_NNZSUM)
// for the caller's read-back instead of being read here.
struct CodeStepFused {
    bool want_stats = false;
    Lists lists{};                  // out: the final lists of the step (capacities from the selection)
    unsigned long long nsel = 0;    // out: |S|, the total capacity of the lists
    double Lz = 0.0, eta = 0.0;     // out
};

// The handle's side streams (a second and a third, default priority) and their
// events, created on first use; null (and the caller runs everything in order on
// the handle's stream) if they cannot be made.
static hipStream_t side_stream(csc_ctx *h) {
    if (h->side || h->side_failed) return h->side;
    bool ok = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess;
    for (auto &e : h->side_ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&h->side2, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->side2_ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        if (h->side) hipStreamDestroy(h->side);
        if (h->side2) hipStreamDestroy(h->side2);
        for (auto &e : h->side_ev)
            if (e) hipEventDestroy(e);
        if (h->side2_ev) hipEventDestroy(h->side2_ev);
        h->side = h->side2 = nullptr;
        for (auto &e : h->side_ev) e = nullptr;
        h->side2_ev = nullptr;
        h->side_failed = true;
    }
    return h->side;
}

// The code update of csc_code_step; hold: the unselected coordinates keep their
// values (csc_code_step_hold).  Their codes enter every residual through
// x_eff = x - D z_held, formed once, and only the sample is written back.
int code_step_impl(csc_ctx *h, const csc_images *im, const float *x, const uint8_t *W, const float *d, int K, int m,
                   float *z, double lambda, double p, uint64_t seed, uint32_t draw, int n_iter, double step,
                   int precision, csc_code_stats *stats, bool hold, CodeStepFused *fo = nullptr) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!x || !d || (!z && !fo)) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z}))) return st;
    if (fo && hold) return fail(h, CSC_EINVAL, "a fused code step starts from zero codes");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(h, CSC_EINVAL, "lambda must be finite and >= 0");
    if (!(p > 0.0 && p <= 1.0)) return fail(h, CSC_EINVAL, "p must lie in (0, 1]");
    if (n_iter < 0) return fail(h, CSC_EINVAL, "n_iter must be >= 0");
    if (!std::isfinite(step)) return fail(h, CSC_EINVAL, "step must be finite");
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;

    const int W32 = (K + 31) / 32;
    WS(mw, unsigned, WS_MASK, (size_t)W32 * g.n_pix);
    WS(cnt32, unsigned, WS_CNT32, g.n_pix);
    WS(soff, unsigned, WS_OFF, g.n_pix + 1);
    WS(tmp, unsigned long long, WS_SCANTMP, scan_tmp_elems(g.n_pix));
    WS(sc, double, WS_SCAL, SC_COUNT);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(sc + SC_TOTAL);
    const unsigned long long thr = (unsigned long long)std::floor(std::ldexp(p, 32));
    // L_z (when no step is given) and the selection are formed first and read back
    // together, in one round trip; until then only workspace has been written
    if (step <= 0.0) {
        const int P = dft_size(g.max_side, m);
        WS(ltmp, double, WS_LIP, lipschitz_tmp_elems(K, m, P));
        PROF(CSC_PK_LIPSCHITZ);
        HIPCHK(launch_lipschitz_code(d, K, m, P, ltmp, sc + SC_LZ, h->stream));
    }
    {
        PROF(CSC_PK_SELECT);
        HIPCHK(launch_mask_count(g, K, thr, seed, draw, mw, cnt32, h->stream));
        HIPCHK(launch_scan(cnt32, soff, g.n_pix, tmp, total, h->stream));
    }
    // The work that does not depend on the size of the selection is queued before
    // the read-back, so that the GPU has it in hand when the host waits.
    WS(R, float, WS_R, g.n_pix);
    // step and threshold as device scalars (from L_z on the device when no step is
    // given), and the counter of list entries at zero
    unsigned long long *nnzsum = reinterpret_cast<unsigned long long *>(sc + SC_NNZSUM);
    float *ethr = reinterpret_cast<float *>(sc + SC_ETHR);
    HIPCHK(launch_set_step(ethr, sc + SC_LZ, step, lambda, nnzsum, h->stream));
    unsigned short *nzc[2];
    {
        WS(c0, unsigned short, WS_NZC0, g.n_pix);
        WS(c1, unsigned short, WS_NZC1, g.n_pix);
        nzc[0] = c0;
        nzc[1] = c1;
    }
    // codes from zero: every list starts empty
    if (fo) HIPCHK(hipMemsetAsync(nzc[0], 0, sizeof(unsigned short) * g.n_pix, h->stream));
    const float *xi = x, *di = d;
    const uint8_t *Wi = W;
    const bool use_graph = h->graphs && n_iter > 0 &&
                           variant_settled(h, synth_key(h, K, m, SYNTH_RESIDUAL, precision));
    // stable copies of the inputs the graph reads (x_eff is copied once it is formed)
    auto copy_x = [&](const float *xs) -> int {
        WS(xc, float, WS_XC, g.n_pix);
        HIPCHK(hipMemcpyAsync(xc, xs, sizeof(float) * g.n_pix, hipMemcpyDeviceToDevice, h->stream));
        xi = xc;
        return CSC_OK;
    };
    const bool hold_x = hold && n_iter > 0;
    if (use_graph) {
        if (!hold_x && (st = copy_x(x))) return st;
        WS(dc, float, WS_DC, (size_t)K * m * m);
        HIPCHK(hipMemcpyAsync(dc, d, sizeof(float) * K * m * m, hipMemcpyDeviceToDevice, h->stream));
        di = dc;
        if (W) {
            WS(wc, uint8_t, WS_WC, g.n_pix);
            HIPCHK(hipMemcpyAsync(wc, W, g.n_pix, hipMemcpyDeviceToDevice, h->stream));
            Wi = wc;
        }
    }
    __bf16 *sda = nullptr, *ada = nullptr;
    if (precision == CSC_BF16 && n_iter > 0) {
        WS(buf, __bf16, WS_SDA, synth_mfma_prep_elems(K));
        HIPCHK(launch_synth_mfma_prep(di, K, m, buf, h->stream));
        sda = buf;
        WS(abuf, __bf16, WS_ADA, adj_prep_elems(K, m));
        HIPCHK(launch_adj_prep(di, K, m, abuf, h->stream));
        ada = abuf;
    }
    if ((st = read_scalars(h, sc, SC_COUNT))) return st;
    double Lz = 0.0, eta = step;
    if (step <= 0.0) {
        Lz = h->h_pinned[SC_LZ];
        if (!(Lz > 0.0)) return fail(h, CSC_EINVAL, "all filters are zero (L_z = 0); pass an explicit step");
        eta = 1.0 / Lz;
    }
    unsigned long long nsel;
    std::memcpy(&nsel, &h->h_pinned[SC_TOTAL], sizeof(nsel));
    if (nsel >= (1ULL << 32)) return fail(h, CSC_EUNSUPPORTED, "more than 2^32 selected coordinates");
    Pair *pairs[2];
    {
        WS(p0, Pair, WS_PAIRS0, nsel + 1);
        WS(p1, Pair, WS_PAIRS1, nsel + 1);
        pairs[0] = p0;
        pairs[1] = p1;
    }
    if (!fo) {
        PROF(CSC_PK_GATHER);
        HIPCHK(launch_gather_selected(g, K, mw, soff, z, pairs[0], nzc[0], nnzsum, h->stream));
    }
    if (hold_x) {
        // lists of the held codes (non-zero, off the sample), then x_eff = x - D z_held
        WS(hcnt, unsigned, WS_HCNT32, g.n_pix);
        WS(hoff, unsigned, WS_HOFF, g.n_pix + 1);
        {
            PROF(CSC_PK_LISTS);
            HIPCHK(launch_count_held(g, K, mw, z, hcnt, h->stream));
            HIPCHK(launch_scan(hcnt, hoff, g.n_pix, tmp, total, h->stream));
        }
        // capacity: every unselected coordinate when that bound is modest, else the exact count
        unsigned long long hcap = (unsigned long long)K * (unsigned long long)g.n_pix - nsel;
        if (hcap >= (1ULL << 32) || hcap * sizeof(Pair) > LIST_BOUND_BYTES) {
            if ((st = read_scalars(h, sc, SC_COUNT))) return st;
            std::memcpy(&hcap, &h->h_pinned[SC_TOTAL], sizeof(hcap));
            if (hcap >= (1ULL << 32)) return fail(h, CSC_EUNSUPPORTED, "more than 2^32 held codes");
        }
        WS(hp, Pair, WS_HPAIRS, hcap + 1);
        WS(hc, unsigned short, WS_HNZC, g.n_pix);
        WS(xe, float, WS_XE, g.n_pix);
        {
            PROF(CSC_PK_LISTS);
            HIPCHK(launch_fill_held(g, K, mw, z, hoff, hp, hc, h->stream));
        }
        {
            PROF(CSC_PK_SYNTH);
            HIPCHK(synth(h, K, m, Lists{hoff, hc, hp}, d, x, nullptr, xe, SYNTH_RESIDUAL, false, precision));
        }
        if (use_graph) {
            if ((st = copy_x(xe))) return st;
        } else {
            xi = xe;
        }
    }
    // The n_iter iterations only launch kernels; their step and threshold are
    // read from device scalars, so the same launches can be replayed as a graph.
    // one stream: the adjoint that loads a chunk ahead, unless a variant is forced
    // (the forced variant's low bit picks the adjoint, so tests reach both)
    const int adj_variant = h->force_variant >= 0 ? (h->force_variant & 1) : 0;
    auto iterations = [&]() -> int {
        int c = 0;
        for (int it = 0; it < n_iter; ++it) {
            {
                PROF(CSC_PK_SYNTH);
                HIPCHK(synth(h, K, m, Lists{soff, nzc[c], pairs[c]}, di, xi, Wi, R, SYNTH_RESIDUAL, it == n_iter - 1,
                             precision, sda));
            }
            {
                PROF(CSC_PK_ADJOINT);
                if (precision == CSC_BF16)
                    HIPCHK(launch_adjoint_shrink_mfma(g, K, m, mw, soff, pairs[c], nzc[c], pairs[c ^ 1], nzc[c ^ 1],
                                                      R, ada, ethr, nnzsum, adj_variant, h->stream));
                else
                    HIPCHK(launch_adjoint_shrink(g, K, m, mw, soff, pairs[c], nzc[c], pairs[c ^ 1], nzc[c ^ 1], R,
                                                 di, ethr, nnzsum, h->stream));
            }
            c ^= 1;
        }
        return CSC_OK;
    };
    // With eager launches and a tuned synthesis, three parts of the batch (two for
    // two images; split between images, which the iterations never couple) run on
    // the handle's stream and its side streams, so that the kernels of one part
    // fill the CUs that another part's last workgroups leave idle.  Same kernels
    // and tiles as one launch over the batch, so the same bits.  The synthesis and
    // adjoint variants that run best beside each other (variant index =
    // synthesis variant * adjoint variants + adjoint variant; the FP32 adjoint has
    // one) are chosen in two stages: after the first split call's iterations,
    // every pair is timed on its last iteration, repeated five times back to back
    // from the same lists without the non-zero count (which rewrites the same
    // bits); the two fastest, and the loop on one stream without a split, then run
    // the next three calls, whose iteration loops are timed, and the fastest is
    // kept (a caller's sixth call runs the choice).
    const bool bf16 = precision == CSC_BF16;
    const auto skey = synth_key(h, K, m, SYNTH_RESIDUAL, precision);
    hipStream_t hs = (!use_graph && !h->prof && n_iter > 0 && g.n_img >= 2 && h->force_variant < 0 &&
                      tuned_variant(h, skey) >= 0)
                         ? side_stream(h)
                         : nullptr;
    if (hs) {
        // three parts when the batch has three images or more
        const int NPART = g.n_img >= 3 ? 3 : 2;
        Geometry part[3];
        for (int i = 0; i < NPART; ++i) {
            const int t0 = g.h_img[g.n_img * i / NPART].tile_off;
            const int t1 = i + 1 < NPART ? g.h_img[g.n_img * (i + 1) / NPART].tile_off : g.n_tiles;
            part[i].n_img = g.n_img;
            part[i].n_pix = g.n_pix;
            part[i].max_side = g.max_side;
            part[i].d_img = g.d_img;
            part[i].d_tiles = g.d_tiles + t0;
            part[i].n_tiles = t1 - t0;
        }
        const hipStream_t pstr[3] = {h->stream, hs, h->side2};
        const int n_av = bf16 ? 2 : 1;
        const int n_vi = (bf16 ? SYNTH_MFMA_VARIANTS : SYNTH_FP32_VARIANTS) * n_av;
        const std::array<int, 5> ikey = {bf16 ? TK_SPLIT_BF16 : TK_SPLIT_FP32, m, K, ilog2(g.n_pix), 0};
        // one iteration on every part's stream from lists c; acc: the non-zero count, or null
        auto iteration = [&](int vi, int c, unsigned long long *acc) -> hipError_t {
            const int sv = vi / n_av, av = vi % n_av;
            const Lists Lc{soff, nzc[c], pairs[c]};
            hipError_t e = hipSuccess;
            for (int i = 0; i < NPART && e == hipSuccess; ++i)
                e = bf16 ? launch_synth_mfma(part[i], K, m, Lc, sda, xi, Wi, R, (int)SYNTH_RESIDUAL, sv, pstr[i])
                         : launch_synth(part[i], K, m, Lc, di, xi, Wi, R, SYNTH_RESIDUAL, sv, pstr[i]);
            for (int i = 0; i < NPART && e == hipSuccess; ++i)
                e = bf16 ? launch_adjoint_shrink_mfma(part[i], K, m, mw, soff, pairs[c], nzc[c], pairs[c ^ 1],
                                                      nzc[c ^ 1], R, ada, ethr, acc, av, pstr[i])
                         : launch_adjoint_shrink(part[i], K, m, mw, soff, pairs[c], nzc[c], pairs[c ^ 1], nzc[c ^ 1],
                                                 R, di, ethr, acc, pstr[i]);
            return e;
        };
        auto fork = [&]() -> hipError_t {
            hipError_t e = hipEventRecord(h->side_ev[0], h->stream);
            for (int i = 1; i < NPART && e == hipSuccess; ++i) e = hipStreamWaitEvent(pstr[i], h->side_ev[0], 0);
            return e;
        };
        auto join = [&]() -> hipError_t {
            hipEvent_t ev[3] = {nullptr, h->side_ev[3], h->side2_ev};
            hipError_t e = hipSuccess;
            for (int i = 1; i < NPART && e == hipSuccess; ++i) {
                e = hipEventRecord(ev[i], pstr[i]);
                if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, ev[i], 0);
            }
            return e;
        };
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const bool can_tune = h->autotune && hipStreamIsCapturing(h->stream, &cs) == hipSuccess &&
                              cs == hipStreamCaptureStatusNone;
        hipGetLastError();
        int vi = tuned_variant(h, ikey);
        const bool settled = vi >= 0;
        int confirm = -1;  // the candidate this call confirms
        auto stt = h->split_tune.find(ikey);
        if (!settled) {
            vi = n_av * tuned_variant(h, skey);
            if (stt != h->split_tune.end() && can_tune) {
                csc_ctx::SplitTune &t = stt->second;
                if (t.pending >= 0) {
                    float ms = 0.f;
                    HIPCHK(hipEventSynchronize(h->split_ev[1]));
                    HIPCHK(hipEventElapsedTime(&ms, h->split_ev[0], h->split_ev[1]));
                    if (t.ms[t.pending] < 0.f || ms < t.ms[t.pending]) t.ms[t.pending] = ms;
                    t.pending = -1;
                }
                if (t.runs >= 3) {
                    int b = 0;
                    for (int i = 1; i < 3; ++i)
                        if (t.ms[i] < t.ms[b]) b = i;
                    vi = t.cand[b];
                    if (std::getenv("SCSC_TUNE_LOG"))
                        std::fprintf(stderr,
                                     "[scsc tune] split m %d K %d: variant %d %.3f ms, variant %d %.3f ms, "
                                     "one stream %.3f ms\n",
                                     m, K, t.cand[0], t.ms[0], t.cand[1], t.ms[1], t.ms[2]);
                    h->tuned[ikey] = vi;
                    h->split_tune.erase(stt);
                } else {
                    confirm = t.runs++;
                    vi = t.cand[confirm];
                }
            }
        }
        if (confirm >= 0) {
            for (auto &e : h->split_ev)
                if (!e) HIPCHK(hipEventCreate(&e));
            HIPCHK(hipEventRecord(h->split_ev[0], h->stream));
        }
        int c = n_iter & 1;
        if (vi == n_vi) {  // the loop on the handle's stream
            if ((st = iterations())) return st;
        } else {
            HIPCHK(fork());
            c = 0;
            for (int it = 0; it < n_iter; ++it) {
                HIPCHK(iteration(vi, c, nnzsum));
                c ^= 1;
            }
            HIPCHK(join());
        }
        if (confirm >= 0) {
            HIPCHK(hipEventRecord(h->split_ev[1], h->stream));
            h->split_tune[ikey].pending = confirm;
        }
        if (!settled && can_tune && h->split_tune.find(ikey) == h->split_tune.end() && h->tuned.count(ikey) == 0) {
            // screening: every pair on the last iteration, five times back to back
            for (auto &e : h->split_ev)
                if (!e) HIPCHK(hipEventCreate(&e));
            std::vector<std::pair<float, int>> rank;
            for (int v = 0; v < n_vi; ++v) {
                float best = 0.f;
                for (int rep = 0; rep < 3; ++rep) {  // the first run warms up
                    HIPCHK(hipEventRecord(h->split_ev[0], h->stream));
                    HIPCHK(fork());
                    for (int r5 = 0; r5 < 5; ++r5) HIPCHK(iteration(v, c ^ 1, nullptr));
                    HIPCHK(join());
                    HIPCHK(hipEventRecord(h->split_ev[1], h->stream));
                    HIPCHK(hipEventSynchronize(h->split_ev[1]));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, h->split_ev[0], h->split_ev[1]));
                    if (rep == 1 || (rep > 1 && ms < best)) best = ms;
                }
                if (std::getenv("SCSC_TUNE_LOG"))
                    std::fprintf(stderr, "[scsc tune] split m %d K %d screening: variant %d %.1f us\n", m, K, v,
                                 1e3 * best);
                rank.push_back({best, v});
            }
            std::sort(rank.begin(), rank.end());
            csc_ctx::SplitTune t;
            t.cand[0] = rank[0].second;
            t.cand[1] = rank[1].second;
            t.cand[2] = n_vi;  // no split
            h->split_tune[ikey] = t;
        }
    } else if (use_graph) {
        const std::vector<uintptr_t> key = {
            (uintptr_t)K, (uintptr_t)m, (uintptr_t)precision, (uintptr_t)n_iter, (uintptr_t)g.n_tiles,
            (uintptr_t)g.n_pix, (uintptr_t)(h->force_variant + 1), (uintptr_t)tuned_variant(h, synth_key(h, K, m, SYNTH_RESIDUAL, precision)),
            (uintptr_t)g.d_img, (uintptr_t)g.d_tiles, (uintptr_t)mw, (uintptr_t)soff, (uintptr_t)pairs[0],
            (uintptr_t)pairs[1], (uintptr_t)nzc[0], (uintptr_t)nzc[1], (uintptr_t)R, (uintptr_t)sc, (uintptr_t)xi,
            (uintptr_t)di, (uintptr_t)Wi, (uintptr_t)sda, (uintptr_t)ada};
        if ((st = graph_replay(h, 0, key, iterations))) return st;
    } else if ((st = iterations())) {
        return st;
    }
    const int cur = n_iter & 1;
    if (z) {
        PROF(CSC_PK_SCATTER);
        if (hold) HIPCHK(launch_scatter_selected(g, K, mw, Lists{soff, nzc[cur], pairs[cur]}, z, h->stream));
        else HIPCHK(launch_scatter_dense(g, K, Lists{soff, nzc[cur], pairs[cur]}, z, h->stream));
    }
    if (fo) {
        if (fo->want_stats) {
            unsigned long long *nnz = reinterpret_cast<unsigned long long *>(sc + SC_CNNZ);
            HIPCHK(hipMemsetAsync(nnz, 0, sizeof(unsigned long long), h->stream));
            HIPCHK(launch_sum_counts(nzc[cur], g.n_pix, nnz, h->stream));
        }
        fo->lists = Lists{soff, nzc[cur], pairs[cur]};
        fo->nsel = nsel;
        fo->Lz = Lz;
        fo->eta = eta;
        return CSC_OK;
    }
    if (stats) {
        unsigned long long *nnz = reinterpret_cast<unsigned long long *>(sc + SC_NNZ);
        HIPCHK(hipMemsetAsync(nnz, 0, sizeof(unsigned long long), h->stream));
        HIPCHK(launch_sum_counts(nzc[cur], g.n_pix, nnz, h->stream));
        if ((st = read_scalars(h, sc, SC_COUNT))) return st;
        unsigned long long v, vs;
        std::memcpy(&v, &h->h_pinned[SC_NNZ], sizeof(v));
        std::memcpy(&vs, &h->h_pinned[SC_NNZSUM], sizeof(vs));
        stats->sampled = (int64_t)nsel;
        stats->nnz = (int64_t)v;
        // counts written: z^0 (gather) and z^1..z^T; the synthesis consumed z^0..z^{T-1}
        stats->nnz_iter_sum = n_iter > 0 ? (int64_t)(vs - v) : 0;
        stats->L_z = Lz;
        stats->step = eta;
    }
    return CSC_OK;
}

extern "C" int csc_code_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W, const float *d,
                             int K, int m, float *z, double lambda, double p, uint64_t seed, uint32_t draw,
                             int n_iter, double step, int precision, csc_code_stats *stats) {
    return code_step_impl(h, im, x, W, d, K, m, z, lambda, p, seed, draw, n_iter, step, precision, stats, false);
}

extern "C" int csc_code_step_hold(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                                  const float *d, int K, int m, float *z, double lambda, double p, uint64_t seed,
                                  uint32_t draw, int n_iter, double step, int precision, csc_code_stats *stats) {
    return code_step_impl(h, im, x, W, d, K, m, z, lambda, p, seed, draw, n_iter, step, precision, stats, true);
}

// The paper's ADMM code solver (csc_code_step_admm): the same selection as
// csc_code_step, then n_admm iterations of ADMM on the subsampled LASSO with
// S-vectors (kernels_admm.hip); the operator q -> A^T A q + rho q is a weighted
// synthesis of q, the adjoint at S (threshold 0, step 1) and a merge back into
// the S-vector layout.  The operator acts on every image at once; the CG
// scalars are per image (each image's problem is solved on its own, Alg. 1).
extern "C" int csc_code_step_admm(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                                  const float *d, int K, int m, float *z, double lambda, double p, uint64_t seed,
                                  uint32_t draw, int n_admm, int n_cg, double rho, double alpha,
                                  csc_code_stats *stats) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (st) return st;
    if (!x || !d || !z) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z}))) return st;
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(h, CSC_EINVAL, "lambda must be finite and >= 0");
    if (!(p > 0.0 && p <= 1.0)) return fail(h, CSC_EINVAL, "p must lie in (0, 1]");
    if (n_admm < 0 || n_cg < 0) return fail(h, CSC_EINVAL, "n_admm and n_cg must be >= 0");
    if (!std::isfinite(rho)) return fail(h, CSC_EINVAL, "rho must be finite");
    if (rho <= 0.0) rho = 10.0 * lambda;
    if (!(rho > 0.0)) return fail(h, CSC_EINVAL, "rho must be > 0 (rho <= 0 selects 10 lambda, and lambda is 0)");
    if (!(alpha > 0.0 && alpha < 2.0)) return fail(h, CSC_EINVAL, "alpha must lie in (0, 2)");
    if (im->n > 65535) return fail(h, CSC_EUNSUPPORTED, "ADMM: at most 65535 images per call");
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;

    const int W32 = (K + 31) / 32;
    WS(mw, unsigned, WS_MASK, (size_t)W32 * g.n_pix);
    WS(cnt32, unsigned, WS_CNT32, g.n_pix);
    WS(soff, unsigned, WS_OFF, g.n_pix + 1);
    WS(tmp, unsigned long long, WS_SCANTMP, scan_tmp_elems(g.n_pix));
    WS(sc, double, WS_SCAL, SC_COUNT);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(sc + SC_TOTAL);
    const unsigned long long thr = (unsigned long long)std::floor(std::ldexp(p, 32));
    {
        PROF(CSC_PK_SELECT);
        HIPCHK(launch_mask_count(g, K, thr, seed, draw, mw, cnt32, h->stream));
        HIPCHK(launch_scan(cnt32, soff, g.n_pix, tmp, total, h->stream));
    }
    if ((st = read_scalars(h, sc, SC_COUNT))) return st;
    unsigned long long nsel;
    std::memcpy(&nsel, &h->h_pinned[SC_TOTAL], sizeof(nsel));
    if (nsel >= (1ULL << 32)) return fail(h, CSC_EUNSUPPORTED, "more than 2^32 selected coordinates");
    const long long n = (long long)nsel;
    WS(sel, Pair, WS_PAIRS0, nsel + 1);
    WS(selc, unsigned short, WS_NZC0, g.n_pix);
    WS(cl, Pair, WS_PAIRS1, nsel + 1);
    WS(clc, unsigned short, WS_NZC1, g.n_pix);
    WS(pb, Pair, WS_APACK, nsel + 1);
    WS(vec, float, WS_AVEC, 7 * (nsel + 1));
    WS(zc, unsigned short, WS_AZC, g.n_pix);
    WS(dot, double, WS_ADOT, admm_dot_elems(g.n_img) + 3LL * g.n_img + 1);
    WS(seg, unsigned, WS_ASEG, g.n_img + 1);
    WS(Y, float, WS_R, g.n_pix);
    float *zt = vec, *v = zt + (nsel + 1), *u = v + (nsel + 1), *b0 = u + (nsel + 1), *r = b0 + (nsel + 1),
          *q = r + (nsel + 1), *Aq = q + (nsel + 1);
    double *part = dot, *cgs = dot + admm_dot_elems(g.n_img);
    HIPCHK(launch_seg(g, soff, seg, h->stream));
    float *ethr = reinterpret_cast<float *>(sc + SC_ETHR);
    HIPCHK(launch_set2(ethr, 1.0f, 0.0f, h->stream));  // the adjoint at S with step 1, no shrinkage
    HIPCHK(hipMemsetAsync(zc, 0, sizeof(unsigned short) * g.n_pix, h->stream));
    {
        PROF(CSC_PK_GATHER);
        HIPCHK(launch_sel_list(g, K, mw, soff, z, sel, selc, h->stream));
        HIPCHK(launch_unpack(g, soff, sel, sel, selc, zt, h->stream));  // zt = v = z_prev on S
        HIPCHK(launch_unpack(g, soff, sel, sel, selc, v, h->stream));
        HIPCHK(hipMemsetAsync(u, 0, sizeof(float) * n, h->stream));
    }
    const float frho = (float)rho;
    // out = A^T A vin + rho vin, with A = W D M^T
    auto op = [&](const float *vin, float *out) -> int {
        HIPCHK(launch_pack(sel, vin, pb, n, h->stream));
        {
            PROF(CSC_PK_SYNTH);
            HIPCHK(synth(h, K, m, Lists{soff, selc, pb}, d, nullptr, W, Y, SYNTH_WEIGHTED, false, CSC_FP32));
        }
        {
            PROF(CSC_PK_ADJOINT);
            HIPCHK(launch_adjoint_shrink(g, K, m, mw, soff, pb, zc, cl, clc, Y, d, ethr, nullptr, h->stream));
        }
        HIPCHK(launch_unpack(g, soff, sel, cl, clc, out, h->stream));
        HIPCHK(launch_add_scaled(out, vin, frho, n, h->stream));
        return CSC_OK;
    };
    if (n_admm > 0) {
        // b0 = A^T W x: the residual of zero codes is W x
        {
            PROF(CSC_PK_SYNTH);
            HIPCHK(synth(h, K, m, Lists{soff, zc, pb}, d, x, W, Y, SYNTH_RESIDUAL, false, CSC_FP32));
        }
        {
            PROF(CSC_PK_ADJOINT);
            HIPCHK(launch_adjoint_shrink(g, K, m, mw, soff, pb, zc, cl, clc, Y, d, ethr, nullptr, h->stream));
        }
        HIPCHK(launch_unpack(g, soff, sel, cl, clc, b0, h->stream));
    }
    for (int it = 0; it < n_admm; ++it) {
        PROF(CSC_PK_UPDATE);
        if ((st = op(zt, Aq))) return st;
        HIPCHK(launch_cg_init(r, q, b0, v, u, Aq, frho, n, h->stream));
        HIPCHK(launch_cg_dot(g, r, r, seg, part, 0, cgs, h->stream));
        for (int c = 0; c < n_cg; ++c) {
            if ((st = op(q, Aq))) return st;
            HIPCHK(launch_cg_dot(g, q, Aq, seg, part, 1, cgs, h->stream));
            HIPCHK(launch_axpy_alpha(g, zt, q, cgs, seg, 1.f, h->stream));
            HIPCHK(launch_axpy_alpha(g, r, Aq, cgs, seg, -1.f, h->stream));
            HIPCHK(launch_cg_dot(g, r, r, seg, part, 2, cgs, h->stream));
            HIPCHK(launch_cg_dir(g, q, r, cgs, seg, h->stream));
        }
        HIPCHK(launch_admm_update(zt, v, u, (float)alpha, (float)(lambda / rho), n, h->stream));
    }
    {
        PROF(CSC_PK_SCATTER);
        HIPCHK(launch_pack(sel, v, pb, n, h->stream));
        HIPCHK(launch_scatter_dense(g, K, Lists{soff, selc, pb}, z, h->stream));
    }
    if (stats) {
        unsigned long long *nnz = reinterpret_cast<unsigned long long *>(sc + SC_NNZ);
        HIPCHK(hipMemsetAsync(nnz, 0, sizeof(unsigned long long), h->stream));
        HIPCHK(launch_count_nz(v, n, nnz, h->stream));
        if ((st = read_scalars(h, sc, SC_COUNT))) return st;
        unsigned long long cnt;
        std::memcpy(&cnt, &h->h_pinned[SC_NNZ], sizeof(cnt));
        stats->sampled = (int64_t)nsel;
        stats->nnz = (int64_t)cnt;
        stats->nnz_iter_sum = 0;
        stats->L_z = 0.0;
        stats->step = rho;
    }
    return CSC_OK;
}

// The filter step of csc_dict_step from the lists of the non-zero codes: exact
// capacities (offsets = prefix of the lengths), nz an upper bound of their
// total, xp the entries tagged for the lag pass (row stride lag_rows_stride)
// when that pass runs.  The arguments are checked and the geometry is set.
static int dict_step_lists(csc_ctx *h, const float *x, const uint8_t *W, Lists L, unsigned long long nz, const XPair *xp,
                    float *d, int K, int m, csc_surrogate *sur, int n_iter, double step, int n_power, int precision,
                    double *L_d_out) {
    const Geometry &g = h->geo;
    const int M = m * m;
    const bool need_ld = sur || step <= 0.0 || L_d_out;
    const bool lag_pass = !W && (sur || need_ld);
    int st = CSC_OK;
    FmLists F;
    if ((st = build_fm_lists(h, K, L, nz, &F))) return st;
    WS(sc, double, WS_SCAL, SC_COUNT);
    // Online without an observation mask, the increment of B_bar, the corner-ring
    // products and the power iteration for L_d do not depend on what runs beside
    // them: on the side stream, B_bar and the corner products run while the lag
    // sums form, and the power iteration (from R, once formed) beside the band sums
    // and the expansion of C_bar.  (In order on the handle's stream when graphs or
    // per-kernel timing are on.)
    hipStream_t side = (sur && lag_pass && n_power > 0 && !h->graphs && !h->prof) ? side_stream(h) : nullptr;
    const int M_ = M;
    auto b_increment = [&](hipStream_t s) -> int {
        const int nch = corr_chunks(K);
        WS(part, double, WS_CPART, (size_t)nch * K * M_);
        PROF(CSC_PK_CORR);
        HIPCHK(launch_corr_fm(g, K, m, F.off, F.codes, x, W, true, part, s));
        HIPCHK(launch_reduce_partials_f64_add(part, nch, K * M_, sur->B, s));
        return CSC_OK;
    };
    // the corner-ring products go into C_bar with atomics, before its expansion
    auto corner = [&](hipStream_t s) -> int {
        PROF(CSC_PK_SUR_CORNER);
        HIPCHK(launch_surrogate_corner(g, K, m, L, sur->C, s));
        return CSC_OK;
    };
    if (side) HIPCHK(hipEventRecord(h->side_ev[0], h->stream));  // the lists are built
    // Without an observation mask the lag sums R of the batch give both the
    // surrogate increment and the zero-padded normal matrix used for L_d.
    double *Rl = nullptr, *Es = nullptr;
    if (lag_pass) {
        const long long nl = surrogate_lag_elems(K, m);
        {
            WS(rl, double, WS_LAG, nl);
            Rl = rl;
        }
        if (sur) {
            WS(es, double, WS_ES, nl * 4 * (m / 2 > 0 ? m / 2 : 1));
            Es = es;
        }
        WS(lpart, double, WS_LAGPART, surrogate_lag_part_elems(g, K, m));
        PROF(CSC_PK_SUR_LAG);
        // with the side stream, side_ev[1] marks R formed (before the band sums)
        HIPCHK(launch_surrogate_lag(g, K, m, L, xp, F.off, F.codes, lpart, Rl, Es, side ? h->side_ev[1] : nullptr,
                                    h->stream));
    }
    // The host queues the launches that the handle's stream runs next before the
    // side stream's run of small power-iteration launches.
    if (side) {
        HIPCHK(hipStreamWaitEvent(side, h->side_ev[0], 0));
        if ((st = b_increment(side))) return st;
        if ((st = corner(side))) return st;
        HIPCHK(hipEventRecord(h->side_ev[3], side));
    }
    if (need_ld && !side) {
        if (W) st = power_iteration(h, K, m, L, F, W, n_power, precision);
        else st = power_iteration_lag(h, K, m, Rl, n_power, h->stream);
        if (st) return st;
    }
    double Ld = 0.0;
    auto read_ld = [&]() -> int {
        if (sur || L_d_out) {
            int st2 = read_scalars(h, sc, SC_COUNT);
            if (st2) return st2;
            Ld = h->h_pinned[SC_LAM];
        }
        return CSC_OK;
    };
    if (!sur) {
        if ((st = read_ld())) return st;
        if (step > 0.0) {
            double lam = 1.0 / step;
            HIPCHK(hipMemcpyAsync(sc + SC_LAM, &lam, sizeof(double), hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        }
        WS(G, float, WS_G, K * M);
        WS(R, float, WS_R, g.n_pix);
        for (int it = 0; it < n_iter; ++it) {
            {
                PROF(CSC_PK_SYNTH);
                HIPCHK(synth(h, K, m, L, d, x, W, R, SYNTH_RESIDUAL, true, precision));
            }
            st = precision == CSC_BF16 ? filter_corr_bf16(h, K, m, L, R, G) : filter_corr_lists(h, K, m, F, R, G);
            if (st) return st;
            PROF(CSC_PK_UPDATE);
            HIPCHK(launch_batch_update(d, G, sc + SC_LAM, K, M, h->stream));
        }
    } else {
        // The surrogate increments do not depend on L_d: they are queued before its
        // read-back.  Without an observation mask the first product C_bar d of the
        // filter iterations is fused into the expansion (unused when the step turns
        // out to be a projection only).
        const bool fused = !W && n_iter > 0;
        WS(y, double, WS_Y, K * M);
        if (W) {
            PROF(CSC_PK_SUR_ACC);
            HIPCHK(launch_surrogate_blocks(g, K, m, F.off, F.codes, W, sur->C, h->stream));
        } else {
            WS(tab, unsigned short, WS_TAB, (size_t)M * M);
            WS(mvpart, double, WS_PART, surrogate_matvec_partial_elems(K, m));
            if (side) {
                HIPCHK(hipStreamWaitEvent(h->stream, h->side_ev[3], 0));  // the corner products are in
            } else if ((st = corner(h->stream))) {
                return st;
            }
            {
                PROF(CSC_PK_SUR_EXPAND);
                HIPCHK(launch_surrogate_expand(K, m, Rl, Es, tab, sur->C, fused ? d : nullptr, mvpart, y,
                                               h->stream));
            }
        }
        if (side) {
            HIPCHK(hipStreamWaitEvent(side, h->side_ev[1], 0));  // R is formed
            if ((st = power_iteration_lag(h, K, m, Rl, n_power, side))) return st;
            HIPCHK(hipEventRecord(h->side_ev[2], side));  // B_bar and L_d are done
            HIPCHK(hipStreamWaitEvent(h->stream, h->side_ev[2], 0));
        } else if ((st = b_increment(h->stream))) {
            return st;
        }
        if ((st = read_ld())) return st;
        const bool step_d = sur->Ld_sum + Ld > 0.0;
        sur->t += 1;
        sur->Ld_sum += Ld;
        if (step_d) {
            WS(part, double, WS_PART, surrogate_matvec_partial_elems(K, m));
            for (int it = 0; it < n_iter; ++it) {
                if (it > 0 || !fused) {
                    PROF(CSC_PK_SUR_MV);
                    HIPCHK(launch_surrogate_matvec(K, m, sur->C, d, part, y, h->stream));
                }
                PROF(CSC_PK_UPDATE);
                HIPCHK(launch_online_update(d, y, sur->B, sur->Ld_sum, K, M, h->stream));
            }
        } else {
            for (int it = 0; it < n_iter; ++it) HIPCHK(launch_batch_update(d, nullptr, sc + SC_LAM, K, M, h->stream));
        }
    }
    if (L_d_out) *L_d_out = Ld;
    return CSC_OK;
}

extern "C" int csc_dict_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W, const float *z,
                             float *d, int K, int m, csc_surrogate *sur, int n_iter, double step, int n_power,
                             int precision, double *L_d_out) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!x || !d || !z) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z}))) return st;
    if (n_iter < 0) return fail(h, CSC_EINVAL, "n_iter must be >= 0");
    if (n_power < 1) return fail(h, CSC_EINVAL, "n_power must be >= 1");
    if (!std::isfinite(step)) return fail(h, CSC_EINVAL, "step must be finite");
    if (sur && (st = check_aligned(h, {}, {sur->C, sur->B}))) return st;
    if (sur && (!sur->C || !sur->B || sur->t < 0 || !(sur->Ld_sum >= 0.0)))
        return fail(h, CSC_EINVAL, "surrogate: need C, B, t >= 0 and Ld_sum >= 0");
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;
    const bool need_ld = sur || step <= 0.0 || L_d_out;
    const bool lag_pass = !W && (sur || need_ld);
    Lists L;
    unsigned long long nz = 0;
    const XPair *xp = nullptr;
    const unsigned xmul = lag_pass ? lag_rows_stride(g, K, m) : 0u;
    if ((st = build_nonzero_lists(h, K, z, &L, &nz, xmul ? &xp : nullptr, xmul))) return st;
    return dict_step_lists(h, x, W, L, nz, xp, d, K, m, sur, n_iter, step, n_power, precision, L_d_out);
}

// Exact-capacity lists (and the lag pass's tagged entries when xmul != 0) from
// the lists a code step ends with; their capacities sum to cap.  The output
// takes the code step's other pair and length buffers (free once its last
// iteration has run) and offsets of its own.
static int lists_from_code_step(csc_ctx *h, Lists in, int cur, unsigned long long cap, Lists *out,
                                const XPair **xp_out, unsigned xmul) {
    const Geometry &g = h->geo;
    WS(cnt32, unsigned, WS_CNT32, g.n_pix);
    WS(off, unsigned, WS_COFF, g.n_pix + 1);
    WS(tmp, unsigned long long, WS_SCANTMP, scan_tmp_elems(g.n_pix));
    WS(sc, double, WS_SCAL, SC_COUNT);
    WS(pairs, Pair, cur ? WS_PAIRS0 : WS_PAIRS1, cap + 1);
    WS(nzc, unsigned short, cur ? WS_NZC0 : WS_NZC1, g.n_pix);
    XPair *xp = nullptr;
    if (xmul) {
        WS(xpb, XPair, WS_XPAIRS, cap + 1);
        xp = xpb;
    }
    PROF(CSC_PK_LISTS);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(sc + SC_TOTAL);
    HIPCHK(launch_counts_u32(in.cnt, g.n_pix, cnt32, h->stream));
    HIPCHK(launch_scan(cnt32, off, g.n_pix, tmp, total, h->stream));
    HIPCHK(launch_compact_lists(g, in, off, pairs, nzc, xp, xmul, h->stream));
    *out = Lists{off, nzc, pairs};
    *xp_out = xp;
    return CSC_OK;
}

extern "C" int csc_online_step(csc_handle h, const csc_images *im, const float *x, const uint8_t *W, float *d, int K,
                               int m, float *z, double lambda, double p, uint64_t seed, uint32_t draw, int n_iter,
                               double step, int precision, csc_surrogate *sur, int n_dict_iter, int n_power,
                               csc_code_stats *stats, double *L_d_out) {
    if (!h) return CSC_EINVAL;
    if (!sur || !sur->C || !sur->B || sur->t < 0 || !(sur->Ld_sum >= 0.0))
        return fail(h, CSC_EINVAL, "surrogate: need C, B, t >= 0 and Ld_sum >= 0");
    if (int sa = check_aligned(h, {}, {sur->C, sur->B})) return sa;
    if (n_dict_iter < 0) return fail(h, CSC_EINVAL, "n_dict_iter must be >= 0");
    if (n_power < 1) return fail(h, CSC_EINVAL, "n_power must be >= 1");
    CodeStepFused fo;
    fo.want_stats = stats != nullptr;
    int st = code_step_impl(h, im, x, W, d, K, m, z, lambda, p, seed, draw, n_iter, step, precision, nullptr, false,
                            &fo);
    if (st) return st;
    const Geometry &g = h->geo;
    const unsigned xmul = W ? 0u : lag_rows_stride(g, K, m);
    const int cur = n_iter & 1;
    Lists L;
    const XPair *xp = nullptr;
    if ((st = lists_from_code_step(h, fo.lists, cur, fo.nsel, &L, &xp, xmul))) return st;
    double Ld = 0.0;
    // the filter step reads the device scalars back once (L_d), which brings the
    // code statistics along
    if ((st = dict_step_lists(h, x, W, L, fo.nsel, xp, d, K, m, sur, n_dict_iter, 0.0, n_power, precision, &Ld)))
        return st;
    if (L_d_out) *L_d_out = Ld;
    if (stats) {
        unsigned long long v, vs;
        std::memcpy(&v, &h->h_pinned[SC_CNNZ], sizeof(v));
        std::memcpy(&vs, &h->h_pinned[SC_NNZSUM], sizeof(vs));
        stats->sampled = (int64_t)fo.nsel;
        stats->nnz = (int64_t)v;
        stats->nnz_iter_sum = n_iter > 0 ? (int64_t)(vs - v) : 0;
        stats->L_z = fo.Lz;
        stats->step = fo.eta;
    }
    return CSC_OK;
}

extern "C" int csc_objective(csc_handle h, const csc_images *im, const float *x, const uint8_t *W, const float *d,
                             int K, int m, const float *z, double lambda, double *f_out, double *terms_out) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (st) return st;
    if (!x || !d || !z || !f_out) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z}))) return st;
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(h, CSC_EINVAL, "lambda must be finite and >= 0");
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;
    WS(part, double, WS_PART, 2 * (size_t)g.n_tiles);
    WS(sc, double, WS_SCAL, SC_COUNT);
    {
        PROF(CSC_PK_OBJECTIVE);
        HIPCHK(launch_objective(g, K, m, x, W, d, z, part, sc + SC_OBJ, h->stream));
    }
    if ((st = read_scalars(h, sc, SC_COUNT))) return st;
    const double data = h->h_pinned[SC_OBJ], l1 = h->h_pinned[SC_OBJ + 1];
    *f_out = data + lambda * l1;
    if (terms_out) {
        terms_out[0] = data;
        terms_out[1] = l1;
    }
    return CSC_OK;
}

extern "C" int csc_objective_noalloc(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                                     const float *d, int K, int m, const float *z, double lambda, double *f_out,
                                     double *terms_out) {
    static_assert(sizeof(ImgInfo) == 40 && sizeof(TileInfo) == 16, "record sizes stated in scsc.h");
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (st) return st;
    if (!x || !d || !z || !f_out) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z}))) return st;
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(h, CSC_EINVAL, "lambda must be finite and >= 0");
    std::vector<ImgInfo> imgs;
    std::vector<TileInfo> tiles;
    batch_records(im, imgs, tiles);
    const size_t T = tiles.size();
    const size_t b_img = align256(sizeof(ImgInfo) * imgs.size()), b_tiles = align256(sizeof(TileInfo) * T),
                 b_part = align256(2 * sizeof(double) * T);
    const size_t need = b_img + b_tiles + b_part + 256;
    if (need > CSC_NOALLOC_SCRATCH_BYTES)
        return fail(h, CSC_EINVAL,
                    "batch too large for the allocation-free objective: it needs " + std::to_string(need) +
                        " bytes of scratch, the limit is " + std::to_string(CSC_NOALLOC_SCRATCH_BYTES));
    if (!h->scratch) return fail(h, CSC_EHIP, "the address of the device scratch array was not available");
    HIPCHK(hipSetDevice(h->device));
    unsigned char *base = h->scratch;
    Geometry g;
    g.n_img = im->n;
    g.n_tiles = (int)T;
    g.d_img = reinterpret_cast<ImgInfo *>(base);
    g.d_tiles = reinterpret_cast<TileInfo *>(base + b_img);
    double *part = reinterpret_cast<double *>(base + b_img + b_tiles);
    double *terms = reinterpret_cast<double *>(base + b_img + b_tiles + b_part);
    HIPCHK(hipMemcpyAsync(g.d_img, imgs.data(), sizeof(ImgInfo) * imgs.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(g.d_tiles, tiles.data(), sizeof(TileInfo) * T, hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_objective(g, K, m, x, W, d, z, part, terms, h->stream));  // no timing events: they are created lazily
    // the host records stay alive until the stream has drained
    if ((st = read_scalars(h, terms, 2))) return st;
    const double data = h->h_pinned[0], l1 = h->h_pinned[1];
    *f_out = data + lambda * l1;
    if (terms_out) {
        terms_out[0] = data;
        terms_out[1] = l1;
    }
    return CSC_OK;
}

namespace {
// The filters as the BF16 operand of the dense adjoint (written once per layer call).
int adjoint_operand(csc_ctx *h, int K, int m, const float *d, const __bf16 **dA_out) {
    WS(dA, __bf16, WS_ADA, adj_prep_elems(K, m));
    HIPCHK(launch_adj_prep(d, K, m, dA, h->stream));
    *dA_out = dA;
    return CSC_OK;
}

// out = D^T r at every coordinate, FP32 or with BF16 operands (dA from adjoint_operand).
int adjoint_dense(csc_ctx *h, int K, int m, const float *r, const float *d, const __bf16 *dA, float *out) {
    PROF(CSC_PK_DENSE);
    if (dA) HIPCHK(launch_adjoint_dense_mfma(h->geo, K, m, r, dA, out, h->stream));
    else HIPCHK(launch_adjoint_dense(h->geo, K, m, r, d, out, h->stream));
    return CSC_OK;
}

}  // namespace

extern "C" int csc_synthesize(csc_handle h, const csc_images *im, const float *d, int K, int m, const float *z,
                              float *y, int precision) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!d || !z || !y) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {d, z, y}))) return st;
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    Lists L;
    if ((st = build_nonzero_lists(h, K, z, &L))) return st;
    {
        PROF(CSC_PK_SYNTH);
        HIPCHK(synth(h, K, m, L, d, nullptr, nullptr, y, SYNTH_PLAIN, true, precision));
    }
    return CSC_OK;
}

extern "C" int csc_adjoint(csc_handle h, const csc_images *im, const float *d, int K, int m, const float *r, float *g,
                           int precision) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!d || !r || !g) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {d, r, g}))) return st;
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const __bf16 *dA = nullptr;
    if (precision == CSC_BF16 && (st = adjoint_operand(h, K, m, d, &dA))) return st;
    return adjoint_dense(h, K, m, r, d, dA, g);
}

extern "C" int csc_filter_corr(csc_handle h, const csc_images *im, const float *z, int K, int m, const float *r,
                               float *G, int precision) {
    if (!h) return CSC_EINVAL;
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!z || !r || !G) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {z, r, G}))) return st;
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    Lists L;
    unsigned long long nz = 0;
    if ((st = build_nonzero_lists(h, K, z, &L, &nz))) return st;
    if (precision == CSC_BF16) return filter_corr_bf16(h, K, m, L, r, G);
    FmLists F;
    if ((st = build_fm_lists(h, K, L, nz, &F))) return st;
    return filter_corr_lists(h, K, m, F, r, G);
}

// ---------------------------------------------------------------------------
// Unrolled proximal-gradient layer (forward and checkpointed backward)
// ---------------------------------------------------------------------------
namespace {
int check_layer_args(csc_ctx *h, const csc_images *im, int K, int m, int precision, double eta, double lambda) {
    int st = check_images(h, im);
    if (!st) st = check_filters(h, K, m);
    if (!st) st = check_precision(h, precision);
    if (st) return st;
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(h, CSC_EINVAL, "eta must be finite and > 0");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(h, CSC_EINVAL, "lambda must be finite and >= 0");
    return CSC_OK;
}

// Whether a layer's synthesis over the lists just built may tune its launch variant:
// only when they hold a non-zero code (a stack of layers starts from zero codes, on
// which every variant takes the same time, so a choice made there is noise).  The
// count is read back only while the key is still untuned.
int layer_synth_representative(csc_ctx *h, int K, int m, SynthMode mode, int precision, bool *rep) {
    *rep = true;
    if (!h->autotune || h->force_variant >= 0 || h->tuned.count(synth_key(h, K, m, mode, precision))) return CSC_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        hipGetLastError();
        *rep = false;
        return CSC_OK;
    }
    WS(sc, double, WS_SCAL, SC_COUNT);
    int st = read_scalars(h, sc, SC_COUNT);
    if (st) return st;
    unsigned long long nz = 0;
    std::memcpy(&nz, &h->h_pinned[SC_TOTAL], sizeof(nz));
    *rep = nz > 0;
    return CSC_OK;
}

// r = W (x - D z) into R and g = D^T r (dense) into G.
int layer_residual_gradient(csc_ctx *h, int K, int m, const float *x, const uint8_t *W, const float *d,
                            const __bf16 *dA, const float *z, int precision, float **R_out, float **G_out) {
    const Geometry &g = h->geo;
    Lists L;
    int st = build_nonzero_lists(h, K, z, &L);
    if (st) return st;
    bool rep = true;
    if ((st = layer_synth_representative(h, K, m, SYNTH_RESIDUAL, precision, &rep))) return st;
    WS(R, float, WS_R, g.n_pix);
    WS(G, float, WS_DG, (size_t)K * g.n_pix);
    {
        PROF(CSC_PK_SYNTH);
        HIPCHK(synth(h, K, m, L, d, x, W, R, SYNTH_RESIDUAL, rep, precision));
    }
    if ((st = adjoint_dense(h, K, m, R, d, dA, G))) return st;
    *R_out = R;
    *G_out = G;
    return CSC_OK;
}

// G_out = sum_i Z(a)_i^T b_i for dense codes a (lists built here).
int corr_dense(csc_ctx *h, int K, int m, const float *a, const float *b, float *G_out, int precision) {
    Lists L;
    unsigned long long nz = 0;
    int st = build_nonzero_lists(h, K, a, &L, &nz);
    if (st) return st;
    if (precision == CSC_BF16) return filter_corr_bf16(h, K, m, L, b, G_out);
    FmLists F;
    if ((st = build_fm_lists(h, K, L, nz, &F))) return st;
    return filter_corr_lists(h, K, m, F, b, G_out);
}
}  // namespace

extern "C" int csc_ista_forward(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                                const float *d, int K, int m, const uint8_t *mask, const float *z_in, float *z_out,
                                double eta, double lambda, int precision) {
    if (!h) return CSC_EINVAL;
    int st = check_layer_args(h, im, K, m, precision, eta, lambda);
    if (st) return st;
    if (!x || !d || !mask || !z_in || !z_out) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z_in, z_out}))) return st;
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const long long n = (long long)K * h->geo.n_pix;
    const __bf16 *dA = nullptr;
    if (precision == CSC_BF16 && (st = adjoint_operand(h, K, m, d, &dA))) return st;
    float *R = nullptr, *G = nullptr;
    if ((st = layer_residual_gradient(h, K, m, x, W, d, dA, z_in, precision, &R, &G))) return st;
    PROF(CSC_PK_UPDATE);
    HIPCHK(launch_ista_update(n, z_in, G, mask, (float)eta, (float)(eta * lambda), z_out, h->stream));
    return CSC_OK;
}

extern "C" int csc_ista_backward(csc_handle h, const csc_images *im, const float *x, const uint8_t *W,
                                 const float *d, int K, int m, const uint8_t *mask, const float *z_in,
                                 const float *g_out, double eta, double lambda, float *g_z, float *g_d, float *g_x,
                                 int precision) {
    if (!h) return CSC_EINVAL;
    int st = check_layer_args(h, im, K, m, precision, eta, lambda);
    if (st) return st;
    if (!x || !d || !mask || !z_in || !g_out || !g_z || !g_d) return fail(h, CSC_EINVAL, "null pointer argument");
    if ((st = check_aligned(h, {x, d, z_in, g_out, g_z, g_d}))) return st;
    HIPCHK(hipSetDevice(h->device));
    if ((st = geometry(h, im))) return st;
    const Geometry &g = h->geo;
    const int M = m * m;
    const long long n = (long long)K * g.n_pix;
    const float feta = (float)eta;
    // recompute r and u from the layer input, then g_u = g_out on the active selected set
    const __bf16 *dA = nullptr;
    if (precision == CSC_BF16 && (st = adjoint_operand(h, K, m, d, &dA))) return st;
    float *R = nullptr, *G = nullptr;
    if ((st = layer_residual_gradient(h, K, m, x, W, d, dA, z_in, precision, &R, &G))) return st;
    WS(GU, float, WS_GU, (size_t)n);
    {
        PROF(CSC_PK_UPDATE);
        HIPCHK(launch_ista_grad_u(n, z_in, G, mask, g_out, feta, (float)(eta * lambda), GU, h->stream));
    }
    // t = W (D g_u)
    WS(T, float, WS_T, g.n_pix);
    {
        Lists Lu;
        if ((st = build_nonzero_lists(h, K, GU, &Lu))) return st;
        bool rep = true;
        if ((st = layer_synth_representative(h, K, m, SYNTH_WEIGHTED, precision, &rep))) return st;
        PROF(CSC_PK_SYNTH);
        HIPCHK(synth(h, K, m, Lu, d, nullptr, W, T, SYNTH_WEIGHTED, rep, precision));
    }
    // g_d = eta (Z(g_u)^T r - Z(z)^T t)
    WS(G1, float, WS_G, K * M);
    WS(G2, float, WS_W, K * M);
    if ((st = corr_dense(h, K, m, GU, R, G1, precision))) return st;
    if ((st = corr_dense(h, K, m, z_in, T, G2, precision))) return st;
    {
        PROF(CSC_PK_UPDATE);
        HIPCHK(launch_axpby(K * M, feta, G1, -feta, G2, g_d, h->stream));
        if (g_x) HIPCHK(launch_axpby(g.n_pix, feta, T, 0.f, nullptr, g_x, h->stream));
    }
    // g_z = g_u - eta D^T t  (G is free again)
    if ((st = adjoint_dense(h, K, m, T, d, dA, G))) return st;
    PROF(CSC_PK_UPDATE);
    HIPCHK(launch_axpby(n, 1.f, GU, -feta, G, g_z, h->stream));
    return CSC_OK;
}

extern "C" int csc_set_graph(csc_handle h, int enable) {
    if (!h) return CSC_EINVAL;
    h->graphs = enable != 0;
    if (!h->graphs) {
        hipSetDevice(h->device);
        hipStreamSynchronize(h->stream);
        for (int i = 0; i < 2; ++i) {
            if (h->graph_exec[i]) hipGraphExecDestroy(h->graph_exec[i]);
            h->graph_exec[i] = nullptr;
            h->graph_key[i].clear();
        }
    }
    return CSC_OK;
}

extern "C" int csc_set_autotune(csc_handle h, int enable) {
    if (!h) return CSC_EINVAL;
    h->autotune = enable > 0;
    h->force_variant = enable < 0 ? -enable - 1 : -1;
    if (!h->autotune) h->tuned.clear();
    return CSC_OK;
}

extern "C" int csc_profile_enable(csc_handle h, int enable) {
    if (!h) return CSC_EINVAL;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    fold_records(h);
    for (int i = 0; i < CSC_PK_COUNT; ++i) {
        h->prof_launches[i] = 0;
        h->prof_ms[i] = 0.0;
    }
    h->prof = enable != 0;
    return CSC_OK;
}

extern "C" int csc_profile_read(csc_handle h, int kernel_class, int64_t *launches, double *total_ms) {
    if (!h) return CSC_EINVAL;
    if (kernel_class < 0 || kernel_class >= CSC_PK_COUNT || !launches || !total_ms)
        return fail(h, CSC_EINVAL, "profile: bad kernel class or null output");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    fold_records(h);
    *launches = h->prof_launches[kernel_class];
    *total_ms = h->prof_ms[kernel_class];
    return CSC_OK;
}
