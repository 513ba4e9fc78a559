// C ABI of the shift-and-stack library: argument checks, integer shift
// tables, work planning, workspace layout and kernel launches.  Every check
// runs on the host before any HIP call, so a rejected call enqueues nothing.
#include "../../include/sst.h"
#include "sst_internal.h"

#include <algorithm>
#include <new>
#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

using namespace sst;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SST_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int ceil_div(int a, int b) { return (a + b - 1) / b; }

constexpr int kMaxFrames = 65535;
constexpr int kMaxSide = 16384;
constexpr int kMaxGrid = 65535;
constexpr double kMaxShift = 1073741824.0;  // 2^30
// Candidate slots.  Each (tile, row half, velocity) keeps its best kt
// candidates and counts all of them; kt is k_max when the slots of the
// whole grid fit kSlotBudget, else what fits, but at least kKeepMin.  A
// velocity whose kept entries may miss one of its k_max best is recomputed
// exactly after the merge, so kt changes time, never lists.  Velocity-block
// rows whose slots exceed kEntryBudget run in further launches.
constexpr size_t kSlotBudget = size_t(256) << 20;
constexpr int kKeepMin = 4;
constexpr size_t kEntryBudget = size_t(512) << 20;
std::atomic<int> g_keep{0};  // sst_set_slot_keep: cap on kt for plans made from now on (0: none)

int check_dims(int n, int h, int w) {
    if (n < 1 || n > kMaxFrames) return fail(SST_E_ARG, "n = %d frames: need 1..%d", n, kMaxFrames);
    if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide)
        return fail(SST_E_ARG, "frame size %dx%d: need 1..%d per side", w, h, kMaxSide);
    return SST_OK;
}

int check_times(const double* t, int n, double t_ref) {
    if (!t) return fail(SST_E_ARG, "t is NULL");
    if (!std::isfinite(t_ref)) return fail(SST_E_ARG, "t_ref is not finite");
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(t[i])) return fail(SST_E_ARG, "t[%d] is not finite", i);
        if (i > 0 && !(t[i] > t[i - 1]))
            return fail(SST_E_UNSORTED, "timestamps must be strictly increasing (t[%d] <= t[%d])", i, i - 1);
    }
    return SST_OK;
}

int check_grid(const double* v, int nv, const char* name) {
    if (!v) return fail(SST_E_ARG, "%s is NULL", name);
    if (nv < 1 || nv > kMaxGrid) return fail(SST_E_ARG, "%s has %d entries: need 1..%d", name, nv, kMaxGrid);
    for (int a = 0; a < nv; ++a)
        if (!std::isfinite(v[a])) return fail(SST_E_ARG, "%s[%d] is not finite", name, a);
    return SST_OK;
}

// d = llround(v * (t - t_ref)): one float64 subtraction and one product
// (separate statements, no contraction), rounded half away from zero.
int shift_of(double t, double t_ref, double v, long long& d) {
    const double tau = t - t_ref;
    const double p = v * tau;
    if (!(std::fabs(p) < kMaxShift)) return SST_E_RANGE;
    d = std::llround(p);
    return SST_OK;
}

// Shift table for the kernels: [n][ld], ld = nv rounded up to a whole
// velocity block; shifts clamped to [-clamp, clamp] (beyond the frame size a
// sample is outside for every output pixel either way); padding columns
// repeat the last real velocity.
int build_table(const double* t, int n, double t_ref, const double* v, int nv, int ld, int clamp,
                std::vector<int32_t>& out, const char* name) {
    out.assign((size_t)n * ld, 0);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < ld; ++a) {
            const int aa = std::min(a, nv - 1);
            long long d;
            if (shift_of(t[i], t_ref, v[aa], d) != SST_OK)
                return fail(SST_E_RANGE, "|%s[%d] * (t[%d] - t_ref)| >= 2^30 px", name, aa, i);
            d = std::max<long long>(-clamp, std::min<long long>(clamp, d));
            out[(size_t)i * ld + a] = (int32_t)d;
        }
    }
    return SST_OK;
}

struct Plan {
    int op = 0;
    int n = 0, h = 0, w = 0;
    int nvx = 0, nvy = 0, ldx = 0, ldy = 0, nvbx = 0, nvby = 0;
    int step_x = 0, step_y = 0, tiles_x = 0, tiles_y = 0, ntiles = 0, nslot = 0;
    int padL = 0, padT = 0, Wp = 0, Hp = 0;
    bool staged = true;
    int shape = 0, vbx = 0, vby = 0;  // velocity-block shape
    int kt = 0, rows_per_chunk = 0, nchunk = 0;
    std::vector<int32_t> DX, DY;
    std::vector<int32_t> G;  // per velocity block: frame order and staging geometry (ord_stride ints)
    size_t ord_stride = 0;
    // workspace offsets (bytes)
    size_t o_geom = 0, o_tab = 0, o_part = 0, o_b = 0, o_s2 = 0, o_P = 0, o_Pb = 0, o_b32 = 0, o_sdev = 0;
    size_t o_flag = 0, flag_bytes = 0;  // list of velocities to recompute (detect)
    size_t o_redo = 0;  // work items left to the second pass (detect, shape 2): counts and marks
    size_t o_ix = 0, o_iy = 0, o_pad = 0, o_tcount = 0, o_ent = 0, o_qpart = 0, o_dt = 0, total = 0;
};

size_t take(size_t& cur, size_t bytes) {
    const size_t o = cur;
    cur = align_up(cur + bytes, 256);
    return o;
}

int make_plan_shape(int op, int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx,
                    const double* vy, int nvy, int k_max, Plan& p, int shape) {
    int rc = check_dims(n, h, w);
    if (rc) return rc;
    if (shape < 0 || shape >= kNShapes) return fail(SST_E_ARG, "velocity-block shape %d: need 0..%d", shape, kNShapes - 1);
    p.op = op;
    p.shape = shape;
    p.vbx = shape_vbx(shape);
    p.vby = shape_vby(shape);
    p.n = n;
    p.h = h;
    p.w = w;
    p.nchunk = (int)(((long long)h * w + kStatChunk - 1) / kStatChunk);
    size_t cur = 0;
    if (op == SST_OP_STATS || op == SST_OP_QUANT || op == SST_OP_REFINE) {
        if (op == SST_OP_QUANT) p.o_qpart = take(cur, (size_t)n * p.nchunk * sizeof(float));
        if (op == SST_OP_REFINE) p.o_dt = take(cur, (size_t)n * sizeof(float));
        p.o_part = take(cur, (size_t)n * p.nchunk * 3 * sizeof(double));
        p.o_b = take(cur, (size_t)n * sizeof(double));
        p.o_s2 = take(cur, (size_t)n * sizeof(double));
        p.o_P = take(cur, (size_t)(n + 1) * sizeof(double));
        p.o_b32 = take(cur, (size_t)n * sizeof(float));
        p.total = cur;
        return SST_OK;
    }
    if (op != SST_OP_STACK && op != SST_OP_DETECT) return fail(SST_E_ARG, "unknown op %d", op);
    if ((rc = check_times(t, n, t_ref))) return rc;
    if ((rc = check_grid(vx, nvx, "vx"))) return rc;
    if ((rc = check_grid(vy, nvy, "vy"))) return rc;
    if (op == SST_OP_DETECT && (k_max < 1 || k_max > kMaxK))
        return fail(SST_E_ARG, "k_max = %d: need 1..%d", k_max, kMaxK);
    const bool detect = op == SST_OP_DETECT;
    p.nvx = nvx;
    p.nvy = nvy;
    p.nvbx = ceil_div(nvx, p.vbx);
    p.nvby = ceil_div(nvy, p.vby);
    p.ldx = p.nvbx * p.vbx;
    p.ldy = p.nvby * p.vby;
    if ((rc = build_table(t, n, t_ref, vx, nvx, p.ldx, w, p.DX, "vx"))) return rc;
    if ((rc = build_table(t, n, t_ref, vy, nvy, p.ldy, h, p.DY, "vy"))) return rc;

    // tiles do not overlap (the peak test of a tile's border pixels
    // evaluates their outside neighbours directly)
    p.step_x = kTileW;
    p.step_y = kRows;
    p.tiles_x = ceil_div(w, p.step_x);
    p.tiles_y = ceil_div(h, p.step_y);
    p.ntiles = p.tiles_x * p.tiles_y;
    p.nslot = 2 * p.ntiles;  // one candidate slot per (tile, row half)

    int dxmin = 0, dxmax = 0, dymin = 0, dymax = 0, sx = 0;
    for (int i = 0; i < n; ++i) {
        const int32_t* rx = &p.DX[(size_t)i * p.ldx];
        for (int a0 = 0; a0 < p.ldx; a0 += p.vbx) {
            const auto mm = std::minmax_element(rx + a0, rx + a0 + p.vbx);
            dxmin = std::min(dxmin, *mm.first);
            dxmax = std::max(dxmax, *mm.second);
            sx = std::max(sx, *mm.second - *mm.first);
        }
        const int32_t* ry = &p.DY[(size_t)i * p.ldy];
        const auto mm = std::minmax_element(ry, ry + p.ldy);
        dymin = std::min(dymin, *mm.first);
        dymax = std::max(dymax, *mm.second);
    }
    // the staged window is CW columns wide: the tile plus the x-shift spread
    // of a block
    const int CW = shape_cw_max(shape);
    p.staged = sx <= CW - kTileW;
    // zero padding so that every staged or direct read stays inside the copy
    const int X0max = (p.tiles_x - 1) * p.step_x;
    const int Y0max = (p.tiles_y - 1) * p.step_y;
    p.padL = std::max(0, -dxmin);
    p.padT = std::max(0, -dymin);
    // columns: a staged window runs CW columns from the tile origin plus the
    // block's smallest shift; rows: kRG row groups from the row group of the
    // pair's smaller y shift; the direct path reads up to the largest shift
    // plus the tile; the frame itself lies inside
    const int need_w = std::max(X0max + std::max(dxmax, 0) + CW, w) + p.padL;
    const int need_h = std::max(Y0max + std::max(dymax, 0) + 4 * kRG + 4, h) + p.padT;
    p.Wp = need_w;
    p.Hp = (int)align_up((size_t)need_h, 4);
    // the staged path addresses each padded frame with 31-bit byte offsets;
    // larger padded frames (shifts of thousands of pixels on large frames)
    // take the direct path, which uses 64-bit addresses
    if ((size_t)p.Hp * (size_t)p.Wp * sizeof(float) > (size_t)0x7FFFFFFF) p.staged = false;
    // Frame order and staging geometry of every velocity block (the same for
    // all tiles: tile origins are multiples of 4 rows).  For frame i the
    // pair's first rows sit at e0, e1 (shift + padT); the window starts at row
    // group gy = min(e0, e1) / 4, and the read pattern is (f0, f1) = (e0, e1) -
    // 4 gy when they are within 4 rows, else two separate reads at row groups
    // G0, G1 past gy with phases e0 % 4, e1 % 4.  Frames are sorted by pattern
    // (stable: ascending i within one); each block holds the frame count of
    // every pattern, then per frame in that order its record: i, window byte
    // offset in the frame (tile origin excluded), G0, G1, and the window
    // column of each x velocity of the block.
    const int rec_ints = shape_rec_ints(shape);
    p.ord_stride = (size_t)kCountInts + (size_t)(n + kRecPad) * rec_ints;
    p.G.assign((size_t)p.nvbx * p.nvby * p.ord_stride, 0);
    std::vector<int> cas(n);
    std::vector<int> order(n);
    for (int by = 0; by < p.nvby && rc == SST_OK; ++by)
        for (int bx = 0; bx < p.nvbx; ++bx) {
            int32_t* blk = &p.G[((size_t)by * p.nvbx + bx) * p.ord_stride];
            for (int i = 0; i < n; ++i) {
                const int32_t* ry = &p.DY[(size_t)i * p.ldy + (size_t)by * kVYW];
                const int e0 = ry[0] + p.padT, e1 = ry[1] + p.padT;
                const int gy = std::min(e0, e1) >> 2;
                const int f0 = e0 - 4 * gy, f1 = e1 - 4 * gy;
                if (std::abs(f1 - f0) <= 4) {
                    cas[i] = std::min(f0, f1) * 9 + (f1 - f0 + 4);
                } else {
                    cas[i] = kNShared + (e0 & 3) * 4 + (e1 & 3);
                    // a separate read must end inside the shape's window
                    if (std::max((e0 >> 2) - gy, (e1 >> 2) - gy) > shape_max_sep(shape)) p.staged = false;
                }
                blk[cas[i]]++;
            }
            for (int i = 0; i < n; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return cas[u] < cas[v]; });
            for (int k = 0; k < n + kRecPad; ++k) {
                const int i = order[std::min(k, n - 1)];
                const int32_t* rx = &p.DX[(size_t)i * p.ldx + (size_t)bx * p.vbx];
                const int32_t* ry = &p.DY[(size_t)i * p.ldy + (size_t)by * kVYW];
                const int mx = *std::min_element(rx, rx + p.vbx);
                const int e0 = ry[0] + p.padT, e1 = ry[1] + p.padT;
                const int gy = std::min(e0, e1) >> 2;
                int32_t* r = &blk[kCountInts + (size_t)k * rec_ints];
                // r[0], r[1]: the frame's address, written with the workspace
                // address when the tables are uploaded
                // (meaningful on the staged path only, where it is below 2^31)
                r[2] = (int32_t)((((long long)gy * p.Wp + mx + p.padL) * 16) & 0x7FFFFFFF);
                const int g0 = cas[i] >= kNShared ? (e0 >> 2) - gy : 0;
                const int g1 = cas[i] >= kNShared ? (e1 >> 2) - gy : 0;
                r[3] = (int32_t)((unsigned)(g0 & 0xFFFF) | ((unsigned)(g1 & 0xFFFF) << 16));
                r[4] = i;
                for (int j = 0; j < p.vbx; ++j) r[kRecCol + j] = rx[j] - mx;
            }
        }

    p.o_tab = take(cur, ((size_t)n * p.ldx + (size_t)n * p.ldy) * sizeof(int32_t));
    p.o_geom = take(cur, p.G.size() * sizeof(int32_t));
    if (detect) {
        // (uploaded as zeros with the tables: the list starts empty, and
        // each run's recomputation leaves it empty)
        p.flag_bytes = ((size_t)kFlagHead + (size_t)p.ldy * nvx) * sizeof(int32_t);
        p.o_flag = take(cur, p.flag_bytes);
    }
    p.o_b32 = take(cur, (size_t)n * sizeof(float));
    p.o_ix = take(cur, (size_t)nvx * w * 2 * sizeof(int32_t));
    p.o_iy = take(cur, (size_t)nvy * h * 2 * sizeof(int32_t));
    p.o_pad = take(cur, (size_t)n * p.Hp * p.Wp * sizeof(float));
    if (detect) {
        p.o_part = take(cur, (size_t)n * p.nchunk * 3 * sizeof(double));
        p.o_b = take(cur, (size_t)n * sizeof(double));
        p.o_s2 = take(cur, (size_t)n * sizeof(double));
        p.o_P = take(cur, (size_t)(n + 1) * sizeof(double));
        p.o_Pb = take(cur, (size_t)(n + 1) * sizeof(double));
        p.o_sdev = take(cur, (size_t)n * 2 * sizeof(double));
        const size_t per_kept = (size_t)p.ldy * nvx * p.nslot * sizeof(Entry);  // one entry in every slot
        p.kt = (int)std::max<size_t>(kKeepMin, std::min<size_t>(k_max, kSlotBudget / per_kept));
        p.kt = std::min(p.kt, k_max);
        if (g_keep.load() > 0) p.kt = std::min(p.kt, g_keep.load());
        const size_t per_row = (size_t)p.vby * nvx * p.nslot * ((size_t)p.kt * sizeof(Entry) + sizeof(int32_t));
        // as few launches as the budget allows, with their rows balanced
        const int max_rows = (int)std::max<size_t>(1, std::min<size_t>(p.nvby, kEntryBudget / per_row));
        const int nchunks = (p.nvby + max_rows - 1) / max_rows;
        p.rows_per_chunk = (p.nvby + nchunks - 1) / nchunks;
        const size_t nk = (size_t)p.rows_per_chunk * p.vby * nvx;
        p.o_tcount = take(cur, nk * p.nslot * sizeof(int32_t));
        p.o_ent = take(cur, nk * p.nslot * p.kt * sizeof(Entry));
        if (shape_split(shape)) {
            const size_t items = (size_t)p.tiles_x * p.tiles_y * shape_items_per_tile(shape) * p.nvbx * p.rows_per_chunk;
            // counts, marks, the list and a count per kCompactChunk marks
            p.o_redo = take(cur, (kRedoHead + 2 * items + items / kCompactChunk + 1) * sizeof(int32_t));
        }
    }
    p.total = cur;
    return SST_OK;
}

constexpr int kShapeAuto = -1;
std::atomic<int> g_stack_shape{kShapeAuto};  // sst_set_stack_shape
std::atomic<int> g_two_pass{SST_TWO_PASS_AUTO};  // sst_set_two_pass

// make_plan_shape with the work-item shape given, or (kShapeAuto) the first
// shape in order of preference whose window holds the grid's shift spread
// (the direct path with the first if none does).  Shape 2 comes first: its
// plain-stack kernel fits four workgroups per CU, and its search waits at a
// barrier every second frame (a tuner may still prefer shape 0 for
// searches that list millions of candidates, whose border pixels shape 2
// evaluates on their own twice as often).
int make_plan(int op, int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx,
              const double* vy, int nvy, int k_max, Plan& p, int shape = kShapeAuto) {
    if (shape == kShapeAuto && op == SST_OP_STACK) shape = g_stack_shape.load();
    if (shape != kShapeAuto) return make_plan_shape(op, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, p, shape);
    static_assert(kNShapes == 3, "an order of preference over every shape");
    static const int order[kNShapes] = {2, 0, 1};
    int rc = make_plan_shape(op, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, p, order[0]);
    if (rc || p.staged || (op != SST_OP_STACK && op != SST_OP_DETECT)) return rc;
    for (int j = 1; j < kNShapes; ++j) {
        Plan q;
        if (make_plan_shape(op, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, q, order[j]) == SST_OK && q.staged) {
            p = std::move(q);
            break;
        }
    }
    g_err.clear();
    return SST_OK;
}

int check_frames(const void* frames, int dtype, const float* scale) {
    if (!frames) return fail(SST_E_ARG, "frames is NULL");
    if (dtype == SST_BF16 || dtype == SST_F16) {
        if (!scale) return fail(SST_E_ARG, "16-bit frames need a per-frame scale array");
        return SST_OK;
    }
    if (dtype != SST_F32) return fail(SST_E_ARG, "unknown frame dtype %d", dtype);
    return SST_OK;
}

int check_ws(const Plan& p, void* ws, size_t ws_bytes) {
    if (!ws) return fail(SST_E_WORKSPACE, "workspace is NULL (need %zu bytes)", p.total);
    if (ws_bytes < p.total) return fail(SST_E_WORKSPACE, "workspace has %zu bytes, need %zu", ws_bytes, p.total);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(SST_E_WORKSPACE, "workspace must be 256-byte aligned");
    return SST_OK;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Pinned staging buffer of the one-shot calls' table uploads: one per
// process, grown when needed, reused once the stream has consumed the last
// copy from it (an event marks that), so a call does not wait for its own
// upload.
struct Staging {
    std::mutex mu;
    void* host = nullptr;
    size_t bytes = 0;
    int device = -1;
    hipEvent_t done = nullptr;
    bool pending = false;
};
Staging g_stage;

// Copy bytes from src to device dst on stream s through the pinned staging
// buffer; returns false (nothing enqueued) if it cannot be used.
bool upload_pinned(const void* src, size_t bytes, void* dst, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_stage.mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (g_stage.device != dev) {
        // (first use, or another device: start over on this one)
        if (g_stage.pending && hipEventSynchronize(g_stage.done) != hipSuccess) return false;
        if (g_stage.done) (void)hipEventDestroy(g_stage.done);
        if (g_stage.host) (void)hipHostFree(g_stage.host);
        g_stage.host = nullptr;
        g_stage.bytes = 0;
        g_stage.done = nullptr;
        g_stage.pending = false;
        if (hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming) != hipSuccess) {
            g_stage.done = nullptr;
            return false;
        }
        g_stage.device = dev;
    }
    if (g_stage.pending) {
        if (hipEventSynchronize(g_stage.done) != hipSuccess) return false;
        g_stage.pending = false;
    }
    if (bytes > g_stage.bytes) {
        if (g_stage.host) (void)hipHostFree(g_stage.host);
        g_stage.host = nullptr;
        g_stage.bytes = 0;
        if (hipHostMalloc(&g_stage.host, bytes, hipHostMallocDefault) != hipSuccess) {
            g_stage.host = nullptr;
            return false;
        }
        g_stage.bytes = bytes;
    }
    std::memcpy(g_stage.host, src, bytes);
    if (hipMemcpyAsync(dst, g_stage.host, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipEventRecord(g_stage.done, s) != hipSuccess) {
        // (the copy is enqueued: wait for it before the buffer is reused)
        (void)hipStreamSynchronize(s);
        return true;
    }
    g_stage.pending = true;
    return true;
}

// Upload the shift tables (and optional per-frame floats) in one copy.
// pinned: through the pinned staging buffer, without waiting (the tables
// are consumed on stream s only); else from pageable memory, waiting for the
// copy (no host allocation: the entry point that allocates nothing).
int upload_tables(const Plan& p, const double* bg, void* ws, hipStream_t s, bool pinned) {
    const size_t nx = (size_t)p.n * p.ldx, ny = (size_t)p.n * p.ldy;
    std::vector<char> host(p.o_b32 - p.o_tab + (size_t)p.n * sizeof(float), 0);
    std::memcpy(host.data(), p.DX.data(), nx * sizeof(int32_t));
    std::memcpy(host.data() + nx * sizeof(int32_t), p.DY.data(), ny * sizeof(int32_t));
    std::memcpy(host.data() + (p.o_geom - p.o_tab), p.G.data(), p.G.size() * sizeof(int32_t));
    {
        // each frame record's padded-copy address in this workspace
        int32_t* g = reinterpret_cast<int32_t*>(host.data() + (p.o_geom - p.o_tab));
        const int rec_ints = shape_rec_ints(p.shape);
        const uintptr_t pad = reinterpret_cast<uintptr_t>(ws) + p.o_pad;
        const size_t fbytes = (size_t)p.Hp * p.Wp * sizeof(float);
        for (size_t b = 0; b < (size_t)p.nvbx * p.nvby; ++b)
            for (int k = 0; k < p.n + kRecPad; ++k) {
                int32_t* r = g + b * p.ord_stride + kCountInts + (size_t)k * rec_ints;
                const uint64_t a = (uint64_t)pad + (uint64_t)r[4] * fbytes;
                r[0] = (int32_t)(uint32_t)(a & 0xFFFFFFFFu);
                r[1] = (int32_t)(uint32_t)(a >> 32);
            }
    }
    size_t bytes = (p.o_flag ? p.o_flag + p.flag_bytes : p.o_geom + p.G.size() * sizeof(int32_t)) - p.o_tab;
    if (bg) {
        float* f = reinterpret_cast<float*>(host.data() + (p.o_b32 - p.o_tab));
        for (int i = 0; i < p.n; ++i) f[i] = (float)bg[i];
        bytes = host.size();
    }
    if (pinned && upload_pinned(host.data(), bytes, at<char>(ws, p.o_tab), s)) return SST_OK;
    (void)hipGetLastError();  // (a failed pinned path falls back to the pageable copy)
    hipError_t e = hipMemcpyAsync(at<char>(ws, p.o_tab), host.data(), bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(shift tables)");
    // the copy is from pageable memory; make sure it has been consumed before
    // `host` goes out of scope
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(shift tables)");
    return SST_OK;
}

StackArgs stack_args(const Plan& p, void* ws) {
    StackArgs a{};
    a.pad = at<float>(ws, p.o_pad);
    a.fstride = (long long)p.Hp * p.Wp;
    a.n = p.n;
    a.h = p.h;
    a.w = p.w;
    a.Wp = p.Wp;
    a.padL = p.padL;
    a.padT = p.padT;
    a.ord = at<int>(ws, p.o_geom);
    a.ord_stride = (long long)p.ord_stride;
    a.cw = shape_cw_max(p.shape);
    a.ni = shape_ni_max(p.shape);
    a.DX = at<int>(ws, p.o_tab);
    a.DY = at<int>(ws, p.o_tab + (size_t)p.n * p.ldx * sizeof(int32_t));
    a.ldx = p.ldx;
    a.ldy = p.ldy;
    a.nvx = p.nvx;
    a.nvy = p.nvy;
    a.IX = at<int>(ws, p.o_ix);
    a.IY = at<int>(ws, p.o_iy);
    a.P = p.o_P ? at<double>(ws, p.o_P) : nullptr;
    a.Pb = p.o_Pb ? at<double>(ws, p.o_Pb) : nullptr;
    a.half = 0;
    a.scale = nullptr;
    a.tiles_x = p.tiles_x;
    a.tiles_y = p.tiles_y;
    a.nvbx = p.nvbx;
    a.vby0 = 0;
    a.nvby = p.nvby;
    a.nslot = p.nslot;
    return a;
}

int prep_and_cov(const Plan& p, const void* frames, int dtype, const float* scale, const float* b32, void* ws,
                 hipStream_t s, bool half = false) {
    PrepArgs pa{};
    pa.half = half ? 1 : 0;
    pa.frames = frames;
    pa.dtype = dtype;
    pa.scale = scale;
    pa.b32 = b32;
    pa.pad = at<float>(ws, p.o_pad);
    pa.n = p.n;
    pa.h = p.h;
    pa.w = p.w;
    pa.Hp = p.Hp;
    pa.Wp = p.Wp;
    pa.padL = p.padL;
    pa.padT = p.padT;
    hipError_t e = launch_prep(pa, s);
    if (e != hipSuccess) return hip_fail(e, "prep kernel");
    const int* DX = at<int>(ws, p.o_tab);
    const int* DY = at<int>(ws, p.o_tab + (size_t)p.n * p.ldx * sizeof(int32_t));
    if ((e = launch_cov(DX, p.ldx, p.n, p.nvx, p.w, at<int>(ws, p.o_ix), s)) != hipSuccess)
        return hip_fail(e, "coverage kernel (x)");
    if ((e = launch_cov(DY, p.ldy, p.n, p.nvy, p.h, at<int>(ws, p.o_iy), s)) != hipSuccess)
        return hip_fail(e, "coverage kernel (y)");
    return SST_OK;
}

// Event pairs around stacking-kernel launches while profiling is on.
constexpr int kProfMax = 4096;
struct Profiler {
    bool on = false;
    int used = 0;
    std::vector<hipEvent_t> ev;  // 2 per launch
    std::mutex mu;
};
Profiler g_prof;

hipError_t launch_stack_profiled(const StackArgs& a, bool detect, bool staged, int shape, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on) return launch_stack(a, detect, staged, shape, s);
    if (g_prof.used >= kProfMax) {
        g_prof.on = false;
        return hipErrorLaunchOutOfResources;
    }
    hipEvent_t e0 = g_prof.ev[2 * g_prof.used], e1 = g_prof.ev[2 * g_prof.used + 1];
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return e;
    e = launch_stack(a, detect, staged, shape, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) ++g_prof.used;
    return e;
}

hipError_t launch_batch_profiled(const BatchArgs& b, int groups, int shape, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on) return launch_stack_batch(b, groups, shape, s);
    if (g_prof.used >= kProfMax) {
        g_prof.on = false;
        return hipErrorLaunchOutOfResources;
    }
    hipEvent_t e0 = g_prof.ev[2 * g_prof.used], e1 = g_prof.ev[2 * g_prof.used + 1];
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return e;
    e = launch_stack_batch(b, groups, shape, s);
    if (e != hipSuccess) return e;
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) ++g_prof.used;
    return e;
}

// The detect launch arguments of a plan for the velocity-block rows
// [r0, r0 + rows).
StackArgs detect_args(const Plan& p, void* ws, float threshold, int min_coverage, int r0, int rows) {
    StackArgs a = stack_args(p, ws);
    a.thr = threshold;
    a.cmin = min_coverage > 0 ? min_coverage : (p.n + 1) / 2;
    a.kt = p.kt;
    a.tcount = at<int32_t>(ws, p.o_tcount);
    a.ent = at<Entry>(ws, p.o_ent);
    a.vby0 = r0;
    a.nvby = rows;
    const long long items = (long long)p.tiles_x * p.tiles_y * shape_items_per_tile(p.shape) * p.nvbx * rows;
    const int mode = g_two_pass.load();
    const bool two = mode == SST_TWO_PASS_ALWAYS || (mode == SST_TWO_PASS_AUTO && items >= kRedoMinItems);
    a.redo = p.o_redo && two ? at<int>(ws, p.o_redo) : nullptr;
    return a;
}

// Whether a detect run of plan p on frames of dtype searches the 16-bit
// samples themselves (IEEE half frames on a staged plan) rather than a
// float32 copy.
std::atomic<int> g_half_search{0};
bool half_search(const Plan& p, int dtype) { return g_half_search.load() != 0 && dtype == SST_F16 && p.staged; }

// Frame statistics, padded copy and coverage intervals of a detect call (and
// for a search on 16-bit samples the frame scales in the records).
int detect_prepare(const Plan& p, void* ws, const void* frames, int dtype, const float* scale, bool stats_out,
                   bool half, hipStream_t s) {
    hipError_t e = launch_stats(frames, dtype, scale, p.n, p.h, p.w, at<double>(ws, p.o_part), p.nchunk,
                                at<double>(ws, p.o_b), at<double>(ws, p.o_s2), at<float>(ws, p.o_b32),
                                at<double>(ws, p.o_P), at<double>(ws, p.o_Pb),
                                stats_out ? at<double>(ws, p.o_sdev) : nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "frame statistics kernels");
    if (half) {
        e = launch_rec_scale(at<int>(ws, p.o_geom), p.nvbx * p.nvby, (long long)p.ord_stride, p.n + kRecPad,
                             shape_rec_ints(p.shape), scale, s);
        if (e != hipSuccess) return hip_fail(e, "record scale kernel");
    }
    return prep_and_cov(p, frames, dtype, scale, at<float>(ws, p.o_b32), ws, s, half);
}

// Merge of the slots of velocity-block rows [r0, r0 + rows) into the lists.
// Workgroups of a recomputation launch (each takes listed velocities until
// none is left; a launch with none listed ends at once).
constexpr int kFixGroups = 512;

// The merge job of velocity-block rows [r0, r0 + rows) of plan p (args: the
// launch's arguments in device memory, or null for the single-plan form).
MergeJob merge_job(const Plan& p, void* ws, int k_max, int r0, int rows, const StackArgs* args) {
    MergeJob J{};
    J.tcount = at<int32_t>(ws, p.o_tcount);
    J.ent = at<Entry>(ws, p.o_ent);
    J.nslot = p.nslot;
    J.kt = p.kt;
    J.k_max = k_max;
    J.nvx = p.nvx;
    J.w = p.w;
    J.k_first = r0 * p.vby * p.nvx;
    J.args = args;
    J.flag = at<int>(ws, p.o_flag);
    J.vbx = p.vbx;
    J.rec = shape_rec_ints(p.shape);
    (void)rows;
    return J;
}

// Merge of the slots of the launch a (velocity-block rows [r0, r0 + rows))
// into the lists, then the exact recomputation of the velocities listed.
int detect_merge(const Plan& p, void* ws, const StackArgs& a, int k_max, int r0, int rows, sst_candidate* cand,
                 int32_t* count, hipStream_t s) {
    const int b_first = r0 * p.vby;
    const int b_last = std::min(p.nvy, (r0 + rows) * p.vby);
    const int nk = (b_last - b_first) * p.nvx;
    hipError_t e = launch_merge(at<int32_t>(ws, p.o_tcount), at<Entry>(ws, p.o_ent), p.nslot, p.kt, k_max, p.nvx,
                                p.w, b_first * p.nvx, nk, cand, count, at<int>(ws, p.o_flag), s);
    if (e != hipSuccess) return hip_fail(e, "merge kernel");
    e = launch_fixup(a, merge_job(p, ws, k_max, r0, rows, nullptr), cand, count, std::min(kFixGroups, nk), s);
    return e != hipSuccess ? hip_fail(e, "recomputation kernel") : SST_OK;
}

// Everything a detect call enqueues after the shift tables are in the
// workspace: kernels only (no host synchronisation, no allocation, no
// memset), so the sequence can be captured into a graph.
int detect_enqueue(const Plan& p, void* ws, const void* frames, int dtype, const float* scale, float threshold,
                   int min_coverage, int k_max, sst_candidate* cand, int32_t* count, bool stats_out, hipStream_t s) {
    int rc;
    const bool half = half_search(p, dtype);
    if ((rc = detect_prepare(p, ws, frames, dtype, scale, stats_out, half, s))) return rc;
    for (int r0 = 0; r0 < p.nvby; r0 += p.rows_per_chunk) {
        const int rows = std::min(p.rows_per_chunk, p.nvby - r0);
        StackArgs a = detect_args(p, ws, threshold, min_coverage, r0, rows);
        if (half) {
            a.half = 1;
            a.scale = scale;
        }
        const hipError_t e = launch_stack_profiled(a, true, p.staged, p.shape, s);
        if (e != hipSuccess) return hip_fail(e, "detect kernel");
        if ((rc = detect_merge(p, ws, a, k_max, r0, rows, cand, count, s))) return rc;
    }
    return SST_OK;
}

}  // namespace

// A prepared detect problem: its geometry and the workspace that holds its
// shift tables.
struct sst_plan {
    Plan p;
    void* ws = nullptr;
    float threshold = 0.f;
    int min_coverage = 0;
    int k_max = 0;
};

// A batch of prepared detect plans whose stacking runs as persistent
// launches: round r covers chunk r (velocity-block rows) of every staged
// plan that has one.  Plans whose blocks are not staged run on their own.
struct sst_batch {
    struct Round {
        std::vector<int> prob;  // plan index of each problem of the round
        BatchArgs args{};
        int groups = 0;
        int shape = 0;  // velocity-block shape of every problem of the round
        int chunk = 0;  // velocity-block-row chunk of every problem
    };
    std::vector<const sst_plan*> plans;
    std::vector<char> solo;
    std::vector<Round> rounds;
    // the staged plans' preparation in groups of at most kPrepMax (plans:
    // their batch indices), and per round the merges likewise
    struct PrepGroup {
        PrepBatch args{};
        int blocks[3] = {0, 0, 0};
        std::vector<int> plans;
    };
    struct MergeGroup {
        MergeBatch args{};
        int blocks = 0;
        std::vector<int> plans;
    };
    std::vector<PrepGroup> prep;
    std::vector<std::vector<MergeGroup>> merges;  // [round]
    // side streams (default priority) over which a run spreads the plans'
    // preparation kernels and merges, forked from and joined to the run's
    // stream by events
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    ~sst_batch() {
        for (int i = 0; i < kSide; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

// Layout of a batch's device tables: per round the problems' arguments, the
// first items and the queue counters.
struct BatchLayout {
    std::vector<int> chunk, shape;  // per launch
    std::vector<size_t> o_tab, o_start, o_cnt;
    std::vector<std::vector<int>> prep_groups;  // staged plans in groups of kPrepMax
    std::vector<size_t> o_pjob, o_poff;         // per group
    std::vector<std::vector<std::vector<int>>> merge_groups;  // [launch][group] plans
    std::vector<std::vector<size_t>> o_mjob, o_moff;
    size_t total = 0;
};

// consecutive groups of at most kPrepMax of the given plan indices
std::vector<std::vector<int>> groups_of(const std::vector<int>& v) {
    std::vector<std::vector<int>> g;
    for (size_t k = 0; k < v.size(); k += kPrepMax)
        g.emplace_back(v.begin() + k, v.begin() + std::min(v.size(), k + (size_t)kPrepMax));
    return g;
}

int plan_chunks(const Plan& p) { return (p.nvby + p.rows_per_chunk - 1) / p.rows_per_chunk; }

// Whether plan p has work in the launch of chunk r and shape sh.
bool in_round(const Plan& p, int r, int sh) { return p.staged && p.shape == sh && r < plan_chunks(p); }

int batch_layout(const sst_plan* const* plans, int nplans, BatchLayout& L) {
    if (!plans || nplans <= 0) return fail(SST_E_ARG, "no plans");
    int rounds = 0;
    for (int j = 0; j < nplans; ++j) {
        if (!plans[j]) return fail(SST_E_ARG, "plan %d is NULL", j);
        if (plans[j]->p.staged) rounds = std::max(rounds, plan_chunks(plans[j]->p));
    }
    size_t cur = 0;
    L = BatchLayout{};
    for (int r = 0; r < rounds; ++r)
        for (int sh = 0; sh < kNShapes; ++sh) {
            int np = 0;
            for (int j = 0; j < nplans; ++j)
                if (in_round(plans[j]->p, r, sh)) ++np;
            if (np == 0) continue;
            L.chunk.push_back(r);
            L.shape.push_back(sh);
            L.o_tab.push_back(take(cur, (size_t)np * sizeof(StackArgs)));
            L.o_start.push_back(take(cur, (size_t)(np + 1) * sizeof(int)));
            L.o_cnt.push_back(take(cur, kBatchQueues * sizeof(int)));
            std::vector<int> in;
            for (int j = 0; j < nplans; ++j)
                if (in_round(plans[j]->p, r, sh)) in.push_back(j);
            L.merge_groups.push_back(groups_of(in));
            L.o_mjob.emplace_back();
            L.o_moff.emplace_back();
            for (const auto& g : L.merge_groups.back()) {
                L.o_mjob.back().push_back(take(cur, g.size() * sizeof(MergeJob)));
                L.o_moff.back().push_back(take(cur, (g.size() + 1) * sizeof(int)));
            }
        }
    std::vector<int> staged;
    for (int j = 0; j < nplans; ++j)
        if (plans[j]->p.staged) staged.push_back(j);
    L.prep_groups = groups_of(staged);
    for (const auto& g : L.prep_groups) {
        L.o_pjob.push_back(take(cur, g.size() * sizeof(PrepJob)));
        L.o_poff.push_back(take(cur, 3 * (g.size() + 1) * sizeof(int)));
    }
    L.total = std::max<size_t>(cur, 256);
    return SST_OK;
}

}  // namespace

extern "C" {

size_t sst_batch_workspace_bytes(const sst_plan* const* plans, int nplans) {
    g_err.clear();
    BatchLayout L;
    return batch_layout(plans, nplans, L) ? 0 : L.total;
}

int sst_batch_create(const sst_plan* const* plans, int nplans, void* ws, size_t ws_bytes, void* stream,
                     sst_batch** batch) {
    g_err.clear();
    if (!batch) return fail(SST_E_ARG, "batch is NULL");
    *batch = nullptr;
    BatchLayout L;
    int rc = batch_layout(plans, nplans, L);
    if (rc) return rc;
    if (!ws || ws_bytes < L.total)
        return fail(SST_E_WORKSPACE, "batch workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SST_E_ARG, "workspace not 256-byte aligned");
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device attributes");
    sst_batch* b = new (std::nothrow) sst_batch;
    if (!b) return fail(SST_E_DEVICE, "out of host memory");
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < sst_batch::kSide && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch streams and events");
    }
    b->plans.assign(plans, plans + nplans);
    b->solo.resize(nplans);
    for (int j = 0; j < nplans; ++j) b->solo[j] = !plans[j]->p.staged;
    std::vector<char> host(L.total, 0);
    b->rounds.resize(L.o_tab.size());
    for (size_t r = 0; r < b->rounds.size(); ++r) {
        auto& R = b->rounds[r];
        R.chunk = L.chunk[r];
        R.shape = L.shape[r];
        std::vector<StackArgs> tab;
        std::vector<int> start(1, 0);
        std::vector<double> cost;  // per item of each problem: frames to add
        for (int j = 0; j < nplans; ++j) {
            const Plan& p = plans[j]->p;
            if (!in_round(p, R.chunk, R.shape)) continue;
            const int r0 = R.chunk * p.rows_per_chunk, rows = std::min(p.rows_per_chunk, p.nvby - r0);
            tab.push_back(detect_args(p, plans[j]->ws, plans[j]->threshold, plans[j]->min_coverage, r0, rows));
            const long long items = (long long)p.tiles_x * p.tiles_y * shape_items_per_tile(p.shape) * p.nvbx * rows;
            if (start.back() + items > 0x7FFFFFFFll) {
                delete b;
                return fail(SST_E_RANGE, "too many work items in one batch round");
            }
            start.push_back(start.back() + (int)items);
            cost.push_back((double)p.n);
            R.prob.push_back(j);
        }
        const int np = (int)R.prob.size();
        // queues of equal cost: problem j's items cost n_j each
        double total = 0.0;
        for (int k = 0; k < np; ++k) total += cost[k] * (start[k + 1] - start[k]);
        R.args.qbegin[0] = 0;
        for (int q = 1; q < kBatchQueues; ++q) {
            const double target = total * q / kBatchQueues;
            double acc = 0.0;
            int item = start[np];
            for (int k = 0; k < np; ++k) {
                const double c = cost[k] * (start[k + 1] - start[k]);
                if (acc + c >= target) {
                    item = start[k] + (int)std::ceil((target - acc) / cost[k]);
                    break;
                }
                acc += c;
            }
            R.args.qbegin[q] = std::max(R.args.qbegin[q - 1], std::min(item, start[np]));
        }
        R.args.qbegin[kBatchQueues] = start[np];
        R.args.tab = at<StackArgs>(ws, L.o_tab[r]);
        R.args.start = at<int>(ws, L.o_start[r]);
        R.args.nprob = np;
        R.args.counter = at<int>(ws, L.o_cnt[r]);
        // as many workgroups as fit on the CUs at once (three per CU of the
        // 4-wave shapes), at least one per queue, the same number per queue
        const int per_cu = kMaxWaves / shape_waves(R.shape);
        const int want = std::max(1, std::min(start[np], std::max(ncu * per_cu, kBatchQueues)));
        R.groups = (want + kBatchQueues - 1) / kBatchQueues * kBatchQueues;
        std::memcpy(host.data() + L.o_tab[r], tab.data(), tab.size() * sizeof(StackArgs));
        std::memcpy(host.data() + L.o_start[r], start.data(), start.size() * sizeof(int));
    }
    // preparation of the staged plans, in groups
    for (size_t g = 0; g < L.prep_groups.size(); ++g) {
        sst_batch::PrepGroup G;
        G.plans = L.prep_groups[g];
        const int np = (int)G.plans.size();
        std::vector<PrepJob> jobs(np);
        std::vector<long long> off(3 * (np + 1), 0);
        for (int k = 0; k < np; ++k) {
            const Plan& p = plans[G.plans[k]]->p;
            void* w = plans[G.plans[k]]->ws;
            PrepJob& J = jobs[k];
            J.part = at<double>(w, p.o_part);
            J.nchunk = p.nchunk;
            J.npx = (long long)p.h * p.w;
            J.b = at<double>(w, p.o_b);
            J.s2 = at<double>(w, p.o_s2);
            J.b32 = at<float>(w, p.o_b32);
            J.P = at<double>(w, p.o_P);
            J.Pb = at<double>(w, p.o_Pb);
            J.pa.b32 = J.b32;
            J.pa.pad = at<float>(w, p.o_pad);
            J.pa.n = p.n;
            J.pa.h = p.h;
            J.pa.w = p.w;
            J.pa.Hp = p.Hp;
            J.pa.Wp = p.Wp;
            J.pa.padL = p.padL;
            J.pa.padT = p.padT;
            J.prep_bx = (int)((((long long)p.Hp / 4) * p.Wp + kStatThreads - 1) / kStatThreads);
            J.DX = at<int>(w, p.o_tab);
            J.DY = at<int>(w, p.o_tab + (size_t)p.n * p.ldx * sizeof(int32_t));
            J.ldx = p.ldx;
            J.ldy = p.ldy;
            J.nvx = p.nvx;
            J.nvy = p.nvy;
            J.w = p.w;
            J.h = p.h;
            J.IX = at<int>(w, p.o_ix);
            J.IY = at<int>(w, p.o_iy);
            off[k + 1] = off[k] + (long long)p.n * p.nchunk;
            off[np + 1 + k + 1] = off[np + 1 + k] + (long long)p.n * J.prep_bx;
            off[2 * (np + 1) + k + 1] = off[2 * (np + 1) + k] +
                                        (long long)(p.w + kStatThreads - 1) / kStatThreads * p.nvx +
                                        (long long)(p.h + kStatThreads - 1) / kStatThreads * p.nvy;
        }
        std::vector<int> off32(off.size());
        for (size_t k = 0; k < off.size(); ++k) {
            if (off[k] > 0x7FFFFFFFll) {
                delete b;
                return fail(SST_E_RANGE, "too many preparation workgroups in one batch group");
            }
            off32[k] = (int)off[k];
        }
        std::memcpy(host.data() + L.o_pjob[g], jobs.data(), jobs.size() * sizeof(PrepJob));
        std::memcpy(host.data() + L.o_poff[g], off32.data(), off32.size() * sizeof(int));
        G.args.jobs = at<PrepJob>(ws, L.o_pjob[g]);
        G.args.off = at<int>(ws, L.o_poff[g]);
        G.args.np = np;
        G.blocks[0] = off32[np];
        G.blocks[1] = off32[2 * np + 1];
        G.blocks[2] = off32[3 * np + 2];
        b->prep.push_back(std::move(G));
    }
    // merges of each round, in groups
    b->merges.resize(b->rounds.size());
    for (size_t r = 0; r < b->rounds.size(); ++r)
        for (size_t g = 0; g < L.merge_groups[r].size(); ++g) {
            sst_batch::MergeGroup M;
            M.plans = L.merge_groups[r][g];
            const int np = (int)M.plans.size();
            std::vector<MergeJob> jobs(np);
            std::vector<int> off(np + 1, 0);
            for (int k = 0; k < np; ++k) {
                const sst_plan* pl = plans[M.plans[k]];
                const Plan& p = pl->p;
                const int r0 = L.chunk[r] * p.rows_per_chunk, rows = std::min(p.rows_per_chunk, p.nvby - r0);
                const int b_first = r0 * p.vby, b_last = std::min(p.nvy, (r0 + rows) * p.vby);
                // (the plan's arguments in this round's table: the merge
                // groups take the round's problems in order)
                const StackArgs* args = at<StackArgs>(ws, L.o_tab[r]) + (g * kPrepMax + k);
                MergeJob& J = jobs[k];
                J = merge_job(p, pl->ws, pl->k_max, r0, rows, args);
                const long long nk = (long long)(b_last - b_first) * p.nvx;
                if (off[k] + nk > 0x7FFFFFFFll) {
                    delete b;
                    return fail(SST_E_RANGE, "too many velocities in one batch merge");
                }
                off[k + 1] = off[k] + (int)nk;
            }
            std::memcpy(host.data() + L.o_mjob[r][g], jobs.data(), jobs.size() * sizeof(MergeJob));
            std::memcpy(host.data() + L.o_moff[r][g], off.data(), off.size() * sizeof(int));
            M.args.jobs = at<MergeJob>(ws, L.o_mjob[r][g]);
            M.args.off = at<int>(ws, L.o_moff[r][g]);
            M.args.np = np;
            M.blocks = off[np];
            b->merges[r].push_back(std::move(M));
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(ws, host.data(), L.total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch table upload");
    }
    *batch = b;
    return SST_OK;
}

int sst_batch_run(const sst_batch* batch, const void* const* frames, const int* dtypes, const float* const* scales,
                  sst_candidate* const* cand, int32_t* const* count, void* stream) {
    g_err.clear();
    if (!batch) return fail(SST_E_ARG, "batch is NULL");
    if (!frames || !dtypes || !cand || !count) return fail(SST_E_ARG, "frames/dtypes/cand/count array is NULL");
    const int np = (int)batch->plans.size();
    int rc;
    for (int j = 0; j < np; ++j) {
        if ((rc = check_frames(frames[j], dtypes[j], scales ? scales[j] : nullptr))) return rc;
        if (!cand[j] || !count[j]) return fail(SST_E_ARG, "cand/count %d is NULL", j);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    constexpr int kS = sst_batch::kSide;
    // fork: work item k goes to stream k mod (kS + 1), stream 0 being s
    auto fork = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(batch->fork, s);
        for (int i = 0; i < kS && e == hipSuccess; ++i) e = hipStreamWaitEvent(batch->side[i], batch->fork, 0);
        return e;
    };
    auto join = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int i = 0; i < kS && e == hipSuccess; ++i) {
            e = hipEventRecord(batch->join[i], batch->side[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, batch->join[i], 0);
        }
        return e;
    };
    hipError_t e;
    // plans too spread for a staged window run on their own, on the side
    // streams, beside the batched work
    bool any_solo = false;
    for (int j = 0; j < np; ++j) any_solo = any_solo || batch->solo[j];
    if (any_solo) {
        if ((e = fork()) != hipSuccess) return hip_fail(e, "batch fork");
        int k = 0;
        for (int j = 0; j < np; ++j) {
            if (!batch->solo[j]) continue;
            const sst_plan* pl = batch->plans[j];
            rc = detect_enqueue(pl->p, pl->ws, frames[j], dtypes[j], scales ? scales[j] : nullptr, pl->threshold,
                                pl->min_coverage, pl->k_max, cand[j], count[j], false, batch->side[k++ % kS]);
            if (rc) return rc;
        }
    }
    // statistics, padded copies and coverage of the staged plans: one launch
    // of each kernel per group
    for (const auto& G : batch->prep) {
        PrepBatch a = G.args;
        for (int k = 0; k < a.np; ++k) {
            const int j = G.plans[k];
            a.frames[k] = frames[j];
            a.dtype[k] = dtypes[j];
            a.scale[k] = scales ? scales[j] : nullptr;
        }
        if ((e = launch_prep_batch(a, G.blocks, s)) != hipSuccess) return hip_fail(e, "batched preparation kernels");
    }
    for (size_t r = 0; r < batch->rounds.size(); ++r) {
        const auto& R = batch->rounds[r];
        if ((e = launch_zero_i32(R.args.counter, kBatchQueues, s)) != hipSuccess)
            return hip_fail(e, "queue reset kernel");
        if ((e = launch_batch_profiled(R.args, R.groups, R.shape, s)) != hipSuccess)
            return hip_fail(e, "batch detect kernel");
        for (const auto& M : batch->merges[r]) {
            MergeBatch a = M.args;
            for (int k = 0; k < a.np; ++k) {
                a.cand[k] = cand[M.plans[k]];
                a.count[k] = count[M.plans[k]];
            }
            if ((e = launch_merge_batch(a, M.blocks, s)) != hipSuccess) return hip_fail(e, "batched merge kernel");
            if ((e = launch_fixup_batch(a, std::min(kFixGroups, M.blocks), s)) != hipSuccess)
                return hip_fail(e, "batched recomputation kernel");
        }
    }
    if (any_solo && (e = join()) != hipSuccess) return hip_fail(e, "batch join");
    return SST_OK;
}

void sst_batch_destroy(sst_batch* batch) { delete batch; }

int sst_set_half_search(int on) { return g_half_search.exchange(on ? 1 : 0); }

int sst_set_stack_shape(int shape, int* previous) {
    g_err.clear();
    if (shape < kShapeAuto || shape >= kNShapes)
        return fail(SST_E_ARG, "work-item shape %d: need -1..%d", shape, kNShapes - 1);
    const int prev = g_stack_shape.exchange(shape);
    if (previous) *previous = prev;
    return SST_OK;
}

int sst_set_two_pass(int mode, int* previous) {
    g_err.clear();
    if (mode < SST_TWO_PASS_NEVER || mode > SST_TWO_PASS_ALWAYS)
        return fail(SST_E_ARG, "two-pass mode %d: need %d..%d", mode, SST_TWO_PASS_NEVER, SST_TWO_PASS_ALWAYS);
    const int prev = g_two_pass.exchange(mode);
    if (previous) *previous = prev;
    return SST_OK;
}

int sst_set_slot_keep(int kt) { return g_keep.exchange(kt > 0 ? kt : 0); }

int sst_profile_begin(void) {
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_prof.mu);
    while ((int)g_prof.ev.size() < 2 * kProfMax) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
        g_prof.ev.push_back(e);
    }
    g_prof.used = 0;
    g_prof.on = true;
    return SST_OK;
}

int sst_profile_end(double* stack_ms, int* stack_launches) {
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const bool overflow = g_prof.on == false && g_prof.used >= kProfMax;
    g_prof.on = false;
    double total = 0.0;
    for (int k = 0; k < g_prof.used; ++k) {
        hipError_t r = hipEventSynchronize(g_prof.ev[2 * k + 1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
        float ms = 0.f;
        r = hipEventElapsedTime(&ms, g_prof.ev[2 * k], g_prof.ev[2 * k + 1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
        total += ms;
    }
    if (stack_ms) *stack_ms = total;
    if (stack_launches) *stack_launches = g_prof.used;
    if (overflow) return fail(SST_E_RANGE, "more than %d profiled launches", kProfMax);
    return SST_OK;
}


const char* sst_last_error(void) { return g_err.c_str(); }

const char* sst_version(void) { return "sst 0.1 (gfx950)"; }

int sst_shift_table(const double* t, int n, double t_ref, const double* v, int nv, int32_t* out) {
    g_err.clear();
    if (n < 1 || n > kMaxFrames) return fail(SST_E_ARG, "n = %d: need 1..%d", n, kMaxFrames);
    int rc = check_times(t, n, t_ref);
    if (rc) return rc;
    if ((rc = check_grid(v, nv, "v"))) return rc;
    if (!out) return fail(SST_E_ARG, "out is NULL");
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < nv; ++a) {
            long long d;
            if (shift_of(t[i], t_ref, v[a], d) != SST_OK)
                return fail(SST_E_RANGE, "|v[%d] * (t[%d] - t_ref)| >= 2^30 px", a, i);
            out[(size_t)i * nv + a] = (int32_t)d;
        }
    return SST_OK;
}

size_t sst_workspace_bytes(int op, int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx,
                           const double* vy, int nvy, int k_max) {
    g_err.clear();
    Plan p;
    if (make_plan(op, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, p) != SST_OK) return 0;
    return p.total;
}

size_t sst_workspace_bytes_shape(int op, int shape, int n, int h, int w, const double* t, double t_ref,
                                 const double* vx, int nvx, const double* vy, int nvy, int k_max) {
    g_err.clear();
    if (shape != kShapeAuto && (shape < 0 || shape >= kNShapes)) {
        fail(SST_E_ARG, "velocity-block shape %d: need 0..%d", shape, kNShapes - 1);
        return 0;
    }
    Plan p;
    if (make_plan(op, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, p, shape) != SST_OK) return 0;
    return p.total;
}

int sst_shape_info(int shape, int* vbx, int* vby) {
    g_err.clear();
    if (shape < 0 || shape >= kNShapes) return fail(SST_E_ARG, "velocity-block shape %d: need 0..%d", shape, kNShapes - 1);
    if (vbx) *vbx = shape_vbx(shape);
    if (vby) *vby = shape_vby(shape);
    return kNShapes;
}

int sst_quantize(const float* frames, int n, int h, int w, int dtype, int center, void* q, float* scale,
                 float* offset, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!frames || !q || !scale) return fail(SST_E_ARG, "frames, q and scale must not be NULL");
    if (dtype != SST_BF16 && dtype != SST_F16) return fail(SST_E_ARG, "quantize: dtype %d is not 16-bit", dtype);
    if (center && !offset) return fail(SST_E_ARG, "quantize: center needs an offset array");
    Plan p;
    int rc;
    if ((rc = make_plan(SST_OP_QUANT, n, h, w, nullptr, 0, nullptr, 0, nullptr, 0, 0, p))) return rc;
    if ((rc = check_ws(p, ws, ws_bytes))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (center) {
        // offset = float32 of each frame's float64 mean (the statistics kernels)
        e = launch_stats(frames, SST_F32, nullptr, n, h, w, at<double>(ws, p.o_part), p.nchunk, at<double>(ws, p.o_b),
                         at<double>(ws, p.o_s2), offset, at<double>(ws, p.o_P), nullptr, nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "frame statistics kernels");
    }
    e = launch_quantize(frames, n, h, w, dtype, center ? offset : nullptr, at<float>(ws, p.o_qpart), p.nchunk, scale,
                        q, s);
    if (e != hipSuccess) return hip_fail(e, "quantize kernels");
    return SST_OK;
}

int sst_refine(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t, double t_ref,
               int n_cand, float* params, int cutout, float fwhm, int steps, float lr, float* snr, float* grad,
               void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_frames(frames, dtype, scale);
    if (rc) return rc;
    if ((rc = check_dims(n, h, w))) return rc;
    if ((rc = check_times(t, n, t_ref))) return rc;
    if (n_cand < 0 || n_cand > (1 << 24)) return fail(SST_E_ARG, "n_cand = %d: need 0..2^24", n_cand);
    if (n_cand > 0 && (!params || !snr)) return fail(SST_E_ARG, "params and snr must not be NULL");
    if (cutout < 1 || cutout > 63 || cutout % 2 == 0) return fail(SST_E_ARG, "cutout = %d: need odd 1..63", cutout);
    if (!(fwhm > 0.f) || !std::isfinite(fwhm)) return fail(SST_E_ARG, "fwhm must be positive and finite");
    if (steps < 0 || steps > 100000) return fail(SST_E_ARG, "steps = %d: need 0..100000", steps);
    if (!std::isfinite(lr)) return fail(SST_E_ARG, "lr is not finite");
    Plan p;
    if ((rc = make_plan(SST_OP_REFINE, n, h, w, nullptr, 0, nullptr, 0, nullptr, 0, 0, p))) return rc;
    if ((rc = check_ws(p, ws, ws_bytes))) return rc;
    if (n_cand == 0) return SST_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_stats(frames, dtype, scale, n, h, w, at<double>(ws, p.o_part), p.nchunk,
                                at<double>(ws, p.o_b), at<double>(ws, p.o_s2), at<float>(ws, p.o_b32),
                                at<double>(ws, p.o_P), nullptr, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "frame statistics kernels");
    std::vector<float> dt(n);
    for (int i = 0; i < n; ++i) dt[i] = (float)(t[i] - t_ref);
    if ((e = hipMemcpyAsync(at<float>(ws, p.o_dt), dt.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(dt)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // PSF: Gaussian of the given FWHM; the sum of its squared weights in float64
    const double sig = (double)fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const int R = cutout / 2;
    double sw2 = 0.0;
    for (int v = -R; v <= R; ++v)
        for (int u = -R; u <= R; ++u) {
            const double wv = std::exp(-(double)(u * u + v * v) / (2.0 * sig * sig));
            sw2 += wv * wv;
        }
    RefineArgs a{};
    a.frames = frames;
    a.dtype = dtype;
    a.scale = scale;
    a.b32 = at<float>(ws, p.o_b32);
    a.P = at<double>(ws, p.o_P);
    a.dt = at<float>(ws, p.o_dt);
    a.n = n;
    a.h = h;
    a.w = w;
    a.params = params;
    a.snr = snr;
    a.grad = grad;
    a.nc = n_cand;
    a.cutout = cutout;
    a.steps = steps;
    a.lr = lr;
    a.inv2s2 = (float)(1.0 / (2.0 * sig * sig));
    a.sw2 = sw2;
    if ((e = launch_refine(a, s)) != hipSuccess) return hip_fail(e, "refine kernel");
    return SST_OK;
}

int sst_median_subtract(const float* frames, int n, int h, int w, float* out, float* median, void* stream) {
    g_err.clear();
    int rc = check_dims(n, h, w);
    if (rc) return rc;
    if (!frames || !out) return fail(SST_E_ARG, "frames and out must not be NULL");
    if (n > kMedianMaxFrames)
        return fail(SST_E_UNSUPPORTED, "median of %d frames: at most %d per call", n, kMedianMaxFrames);
    hipError_t e = launch_median_sub(frames, n, h, w, out, median, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "median kernel");
    return SST_OK;
}

int sst_coadd(const float* frames, int n, int h, int w, int group, float* out, const double* t, double* t_out,
              void* stream) {
    g_err.clear();
    int rc = check_dims(n, h, w);
    if (rc) return rc;
    if (!frames || !out) return fail(SST_E_ARG, "frames and out must not be NULL");
    if (group < 1 || group > n) return fail(SST_E_ARG, "group = %d: need 1..n (%d)", group, n);
    if (t_out && !t) return fail(SST_E_ARG, "t_out needs t");
    const int ng = n / group;
    if (t_out) {
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(t[i])) return fail(SST_E_ARG, "t[%d] is not finite", i);
        for (int g = 0; g < ng; ++g) {
            double acc = 0.0;
            for (int j = 0; j < group; ++j) acc += t[g * group + j];
            t_out[g] = acc / group;
        }
    }
    hipError_t e = launch_coadd(frames, h, w, group, ng, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "co-add kernel");
    return SST_OK;
}

int sst_bin2x2(const float* frames, int n, int h, int w, float* out, void* stream) {
    g_err.clear();
    int rc = check_dims(n, h, w);
    if (rc) return rc;
    if (!frames || !out) return fail(SST_E_ARG, "frames and out must not be NULL");
    if (h < 2 || w < 2) return fail(SST_E_ARG, "binning needs frames of at least 2x2 (got %dx%d)", w, h);
    hipError_t e = launch_bin2x2(frames, n, h, w, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "binning kernel");
    return SST_OK;
}

int sst_frame_stats(const void* frames, int dtype, const float* scale, int n, int h, int w, double* stats, void* ws,
                    size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_frames(frames, dtype, scale);
    if (rc) return rc;
    if (!stats) return fail(SST_E_ARG, "stats is NULL");
    Plan p;
    if ((rc = make_plan(SST_OP_STATS, n, h, w, nullptr, 0, nullptr, 0, nullptr, 0, 0, p))) return rc;
    if ((rc = check_ws(p, ws, ws_bytes))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_stats(frames, dtype, scale, n, h, w, at<double>(ws, p.o_part), p.nchunk,
                                at<double>(ws, p.o_b), at<double>(ws, p.o_s2), at<float>(ws, p.o_b32),
                                at<double>(ws, p.o_P), nullptr, stats, s);
    if (e != hipSuccess) return hip_fail(e, "frame statistics kernels");
    return SST_OK;
}

int sst_stack(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t, double t_ref,
              const double* vx, int nvx, const double* vy, int nvy, const double* bg, int mode, float* out,
              int32_t* cov, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_frames(frames, dtype, scale);
    if (rc) return rc;
    if (!out) return fail(SST_E_ARG, "out is NULL");
    if (mode != SST_SUM && mode != SST_MEAN) return fail(SST_E_ARG, "unknown stack mode %d", mode);
    if (bg)
        for (int i = 0; i < n && i < kMaxFrames; ++i)
            if (!std::isfinite(bg[i])) return fail(SST_E_ARG, "bg[%d] is not finite", i);
    Plan p;
    if ((rc = make_plan(SST_OP_STACK, n, h, w, t, t_ref, vx, nvx, vy, nvy, 0, p))) return rc;
    if ((rc = check_ws(p, ws, ws_bytes))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = upload_tables(p, bg, ws, s, true))) return rc;
    if ((rc = prep_and_cov(p, frames, dtype, scale, bg ? at<float>(ws, p.o_b32) : nullptr, ws, s))) return rc;
    StackArgs a = stack_args(p, ws);
    a.out = out;
    a.cov = cov;
    a.mean = mode == SST_MEAN;
    hipError_t e = launch_stack_profiled(a, false, p.staged, p.shape, s);
    if (e != hipSuccess) return hip_fail(e, "stack kernel");
    return SST_OK;
}

int sst_detect(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t, double t_ref,
               const double* vx, int nvx, const double* vy, int nvy, float threshold, int min_coverage, int k_max,
               sst_candidate* cand, int32_t* count, double* frame_stats, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    return sst::detect_call(frames, dtype, scale, n, h, w, t, t_ref, vx, nvx, vy, nvy, threshold, min_coverage, k_max,
                            cand, count, frame_stats, ws, ws_bytes, stream, true);
}

}  // extern "C"

namespace sst {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int detect_call(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t,
                double t_ref, const double* vx, int nvx, const double* vy, int nvy, float threshold,
                int min_coverage, int k_max, sst_candidate* cand, int32_t* count, double* frame_stats, void* ws,
                size_t ws_bytes, void* stream, bool pinned_upload) {
    int rc = check_frames(frames, dtype, scale);
    if (rc) return rc;
    if (!cand || !count) return fail(SST_E_ARG, "cand/count is NULL");
    if (std::isnan(threshold)) return fail(SST_E_ARG, "threshold is NaN");
    Plan p;
    if ((rc = make_plan(SST_OP_DETECT, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, p))) return rc;
    if ((rc = check_ws(p, ws, ws_bytes))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = upload_tables(p, nullptr, ws, s, pinned_upload))) return rc;
    if ((rc = detect_enqueue(p, ws, frames, dtype, scale, threshold, min_coverage, k_max, cand, count,
                             frame_stats != nullptr, s)))
        return rc;
    if (frame_stats) {
        hipError_t e = hipMemcpyAsync(frame_stats, at<double>(ws, p.o_sdev), (size_t)n * 2 * sizeof(double),
                                      hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(frame stats)");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return SST_OK;
}

}  // namespace sst

extern "C" {

int sst_plan_detect(int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx, const double* vy,
                    int nvy, float threshold, int min_coverage, int k_max, void* ws, size_t ws_bytes, void* stream,
                    sst_plan** plan) {
    return sst_plan_detect_shape(kShapeAuto, n, h, w, t, t_ref, vx, nvx, vy, nvy, threshold, min_coverage, k_max, ws,
                                 ws_bytes, stream, plan);
}

int sst_plan_detect_shape(int shape, int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx,
                          const double* vy, int nvy, float threshold, int min_coverage, int k_max, void* ws,
                          size_t ws_bytes, void* stream, sst_plan** plan) {
    g_err.clear();
    if (shape != kShapeAuto && (shape < 0 || shape >= kNShapes)) {
        if (plan) *plan = nullptr;
        return fail(SST_E_ARG, "velocity-block shape %d: need 0..%d", shape, kNShapes - 1);
    }
    if (!plan) return fail(SST_E_ARG, "plan is NULL");
    *plan = nullptr;
    if (std::isnan(threshold)) return fail(SST_E_ARG, "threshold is NaN");
    sst_plan* pl = new (std::nothrow) sst_plan;
    if (!pl) return fail(SST_E_DEVICE, "out of host memory");
    int rc = make_plan(SST_OP_DETECT, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max, pl->p, shape);
    if (!rc) rc = check_ws(pl->p, ws, ws_bytes);
    if (!rc) rc = upload_tables(pl->p, nullptr, ws, static_cast<hipStream_t>(stream), false);
    if (rc) {
        delete pl;
        return rc;
    }
    pl->ws = ws;
    pl->threshold = threshold;
    pl->min_coverage = min_coverage;
    pl->k_max = k_max;
    *plan = pl;
    return SST_OK;
}

int sst_plan_run(const sst_plan* plan, const void* frames, int dtype, const float* scale, sst_candidate* cand,
                 int32_t* count, void* stream) {
    g_err.clear();
    if (!plan) return fail(SST_E_ARG, "plan is NULL");
    int rc = check_frames(frames, dtype, scale);
    if (rc) return rc;
    if (!cand || !count) return fail(SST_E_ARG, "cand/count is NULL");
    return detect_enqueue(plan->p, plan->ws, frames, dtype, scale, plan->threshold, plan->min_coverage, plan->k_max,
                          cand, count, false, static_cast<hipStream_t>(stream));
}

int sst_plan_info(const sst_plan* plan, int* shape, int* staged, int* launches) {
    g_err.clear();
    if (!plan) return fail(SST_E_ARG, "plan is NULL");
    if (shape) *shape = plan->p.shape;
    if (staged) *staged = plan->p.staged ? 1 : 0;
    if (launches) *launches = plan_chunks(plan->p);
    return SST_OK;
}

void sst_plan_destroy(sst_plan* plan) { delete plan; }

}  // extern "C"
