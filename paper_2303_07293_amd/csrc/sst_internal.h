// Internal declarations shared by the host API (sst_api.cpp) and the HIP
// kernels (sst_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/sst.h"

namespace sst {

// clang vector types (HIP's int4/float4 wrappers are structs that keep
// register arrays of them from being promoted out of scratch)
typedef int i4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Work decomposition of the stack kernels.  A workgroup owns a tile of 64
// columns (one per lane) by kRows rows and a block of VBX x 2 trial
// velocities: one pair of neighbouring y velocities and VBX x velocities, so
// that every staged frame window serves all 2 VBX velocities.  Wave w
// handles the kRowsW = kRows / 2 rows of half w % 2 for kVPW x velocities
// (group w / 2) and both y velocities: kVPW * 2 * kRowsW float accumulators
// per lane.  For one frame the two y velocities sample rows a uniform
// distance apart, so one read of the rows between them feeds both.
constexpr int kWave = 64;
constexpr int kTileW = 64;
constexpr int kRows = 32;
constexpr int kRowsW = kRows / 2;  // rows per wave
constexpr int kVPW = 3;  // x velocities per wave
constexpr int kVYW = 2;  // y velocities per block (one pair)
// Work-item shapes (chosen per plan).  Workgroups of 4 waves, three per CU
// (one waiting at its barrier leaves the SIMDs to the other two; workgroups
// of 6 or 12 waves with windows this size get a CU to themselves and lose
// that).  Shapes 0 and 1: a work item is a whole tile and a block of 6 x
// velocities (waves: 2 row halves x 2 groups of 3 x velocities); they
// differ in the width of the staged window: shape 0 holds an x shift spread
// of 25 px over the block in three ring buffers, shape 1 one of 80 px in two
// (for grids whose shifts grow faster per velocity step).  Shape 2 (tried
// first) splits the tile: a work item is one row half of a tile and a block
// of 12 x velocities (waves: 4 groups of 3), so each staged window is 6 row
// groups high and serves twice as many velocities per row, at the cost of a
// wider x spread (up to 48 px over the block); its search keeps four ring
// buffers and its plain stack runs four workgroups per CU (ring_bufs).  All
// fit the LDS that three workgroups may share.
constexpr int kNShapes = 3;
constexpr int kMaxWaves = 12;  // waves per CU at the kernels' register use
__host__ __device__ constexpr int shape_waves(int) { return 4; }
// work items of shape sh cover one row half of a tile (else the whole tile)
__host__ __device__ constexpr bool shape_split(int sh) { return sh == 2; }
__host__ __device__ constexpr int shape_vbx(int sh) {
    return kVPW * (shape_split(sh) ? shape_waves(sh) : shape_waves(sh) / 2);
}
__host__ __device__ constexpr int shape_vby(int) { return kVYW; }
// work items per tile and velocity block
__host__ __device__ constexpr int shape_items_per_tile(int sh) { return shape_split(sh) ? 2 : 1; }
// LDS staging.  The padded copy of every frame is stored in groups of four
// rows: element (y, x) of a frame at float ((y / 4) * Wp + x) * 4 + y % 4, so
// that one 16-byte chunk holds four consecutive rows of one column.  Per
// frame a window of kRG row groups by cw columns (the tile widened by the
// block's x-shift spread) is staged into LDS with the same layout, and a
// lane reads four rows of its column with one 16-byte LDS read.
constexpr int kRG = 10;  // row groups (40 rows) of the staged window of a whole tile
// row groups of a shape's window: a whole tile, or one row half (16 rows,
// the pair's row spread and a phase fit 6 groups)
__host__ __device__ constexpr int shape_rg(int sh) { return shape_split(sh) ? 6 : kRG; }
__host__ __device__ constexpr int shape_cw_max(int sh) { return sh == 0 ? 89 : (sh == 1 ? 144 : 112); }
__host__ __device__ constexpr int shape_nbuf(int sh) { return sh == 1 ? 2 : 3; }
// Staging buffers of a kernel: four for a kernel that waits at a barrier
// every second frame (pair), else the shape's ring.
__host__ __device__ constexpr int ring_bufs(int sh, bool pair) { return pair ? 4 : shape_nbuf(sh); }
// staging instructions (64 chunks each) of the largest window
__host__ __device__ constexpr int shape_ni_max(int sh) {
    return (shape_rg(sh) * shape_cw_max(sh) + kWave - 1) / kWave;
}
// The same window of 16-bit samples: four rows of a column in 8 bytes, so a
// 16-byte staging chunk holds two columns and the window width is even.
__host__ __device__ constexpr int shape_cw_half(int sh) { return (shape_cw_max(sh) + 1) / 2 * 2; }
__host__ __device__ constexpr int shape_ni_half(int sh) {
    return (shape_rg(sh) * shape_cw_half(sh) / 2 + kWave - 1) / kWave;
}
// Separate reads (below) span 5 row groups from a group offset G past the
// window's first group, plus 4 for the lower half of a whole tile: the
// largest G a shape's window allows
__host__ __device__ constexpr int shape_max_sep(int sh) { return shape_rg(sh) - (shape_split(sh) ? 5 : 9); }
// Frame order.  Within the window the rows of the pair's two y velocities
// start at row offsets f0, f1 of the window's first row group; the pattern
// (f0, f1) of a frame is one of kNCase read cases: 36 where the two start
// within 4 rows of each other (min(f0, f1) in 0..3, f1 - f0 in -4..4; one
// read of the rows between them serves both) and 16 where they are further
// apart (each y velocity read on its own, at its own row group, phases 0..3).
// The host sorts each block's frames by case, and the kernel runs one loop
// per case whose read pattern is fixed at compile time.
constexpr int kNShared = 36;
constexpr int kNCase = kNShared + 16;
constexpr int kCountInts = 64;  // per-block header: frames of each case (kNCase used)
// per-frame record: frame address (2 ints), window byte offset, row-group
// offsets (2 x 16 bits), frame index, the frame's scale (float bits; written
// by each run of a search on 16-bit samples), window column of each x
// velocity
constexpr int kRecScale = 5;
constexpr int kRecCol = 6;
__host__ __device__ constexpr int shape_rec_ints(int sh) { return (kRecCol + shape_vbx(sh) + 3) / 4 * 4; }
// copies of a block's last record after it: the staging ring stages up to
// NBUF - 2 frames past the last and reads the record after those
constexpr int kRecPad = 6;

constexpr int kStatThreads = 256;
constexpr int kStatChunk = 8192;  // pixels per frame-statistics workgroup
constexpr int kMaxK = 1024;       // largest k_max accepted
constexpr int kMergeLds = 2048;   // entries ranked in LDS by the merge kernel
constexpr int kPLds = 256;        // variance-prefix entries the stack kernel keeps in LDS

// One candidate kept by a (tile, velocity) before the per-velocity merge.
struct Entry {
    float sn;
    float flux;
    int32_t raster;
    int32_t cov;
};

// ------------------------------------------------------------ frame values
// Frame value of a stored sample: float32 as is, or a 16-bit sample times
// its frame's scale (one float32 product; the 16-bit to float32 conversion
// is exact).
template <int DT>
__device__ __forceinline__ float frame_value(const void* f, long long e, float sc) {
    if constexpr (DT == SST_F32) {
        return static_cast<const float*>(f)[e];
    } else if constexpr (DT == SST_BF16) {
        const unsigned bits = static_cast<const uint16_t*>(f)[e];
        return sc * __uint_as_float(bits << 16);
    } else {
        return sc * (float)static_cast<const _Float16*>(f)[e];
    }
}

struct StackArgs {
    // zero-padded frames in row groups, [n][Hp/4][Wp][4]: float32 samples
    // minus the frame's background, or (half != 0) the 16-bit samples as
    // stored (IEEE half, frame i at half index 2 i fstride), each multiplied
    // by its frame's scale as it is added, the backgrounds subtracted after
    // the sum through the prefix Pb
    const float* pad;
    long long fstride;  // Hp * Wp floats per frame
    int half;
    const float* scale;  // [n] per-frame scales (half only)
    const double* Pb;    // [n+1] prefix sums of the frame means (half only)
    int n, h, w;
    int Wp, padL, padT;
    // per velocity block [nvby][nvbx]: kCountInts ints (frames of each read
    // case), then per frame in the block's order (and kRecPad copies of the
    // last) a record of rec ints: the frame's padded-copy address (low, high
    // 32 bits), the window byte offset in the frame (tile origin excluded),
    // the row-group offsets of the two y velocities (separate-read cases;
    // 16 bits each), the frame index, and the window column of each x
    // velocity of the block
    const int* ord;
    long long ord_stride;  // ints per block
    int cw;   // window columns
    int ni;   // staging instructions (64 chunks) per frame
    const int* DX;  // [n][ldx] clamped x shifts, columns >= nvx repeat column nvx-1
    const int* DY;  // [n][ldy]
    int ldx, ldy;
    int nvx, nvy;
    const int* IX;    // [nvx][w][2]: first and last frame whose x sample is in the frame
    const int* IY;    // [nvy][h][2]
    const double* P;  // [n+1] prefix sums of the frame variances
    int tiles_x, tiles_y;
    int nvbx;        // velocity blocks along x
    int vby0, nvby;  // velocity-block rows handled by this launch
    // plain stack
    float* out;
    int32_t* cov;
    int mean;
    // detect
    float thr;
    int cmin;
    int kt;      // entries kept per slot
    int nslot;   // slots per velocity: one per (tile, row half), 2 * tiles_x * tiles_y
    int32_t* tcount;  // [velocities of this launch][nslot] candidates found (before keeping kt)
    Entry* ent;       // [velocities of this launch][nslot][kt]
    // (searches of shape 2 in two passes) [kRedoFound]: items the first
    // pass ran that found a pixel above threshold; [kRedoSkipping]: set once
    // the first pass lists every further item without running it;
    // [kRedoTotal]: items listed; [kRedoHead + item]: 1 if the second pass
    // runs the work item; [kRedoHead + G + i]: the i-th such item in order
    // (G: work items of the launch); [kRedoHead + 2 G + c]: marks set among
    // the kCompactChunk items from c kCompactChunk; NULL: one pass
    int* redo;
};

// Two-pass search: once more than one in kRedoSkip of the items dealt so
// far (workgroups are dealt in order) have found a pixel above threshold,
// from the kRedoWarm-th item on, the first pass lists every further item
// for the second without running it. The second pass cuts the list into
// kRedoRuns runs, one per XCD.
constexpr int kRedoRuns = 8;
constexpr int kRedoSkip = 8;
constexpr int kRedoWarm = 2048;
constexpr int kRedoFound = 0;
constexpr int kRedoSkipping = 1;
constexpr int kRedoTotal = 2;
// Launches of fewer work items search in one pass unless two are forced:
// the extra launches cost more than the first pass saves on them.
constexpr int kRedoMinItems = 4096;
constexpr int kRedoHead = 32;
constexpr int kCompactThreads = 1024;  // threads of the workgroups that list the marked items
constexpr int kCompactChunk = 4 * kCompactThreads;  // marks per such workgroup

// One round of a batch of detect problems, run by one persistent launch:
// the arguments of each problem's share of the round, the first global work
// item of each problem, and kBatchQueues queues of consecutive items (one
// per XCD: workgroup g serves queue g mod kBatchQueues, whose items it takes
// one at a time through an atomic counter).
constexpr int kBatchQueues = 8;
struct BatchArgs {
    const StackArgs* tab;  // [nprob]
    const int* start;      // [nprob + 1], start[nprob] = items in the round
    int nprob;
    int* counter;          // [kBatchQueues] items taken, zero before the launch
    int qbegin[kBatchQueues + 1];
};

struct PrepArgs {
    const void* frames;  // [n][h][w] of dtype
    int dtype;           // SST_F32, SST_BF16, SST_F16
    const float* scale;  // [n] per-frame multiplier of 16-bit frames
    const float* b32;    // [n] subtracted per frame, or nullptr
    float* pad;
    int n, h, w, Hp, Wp, padL, padT;
    int half;  // SST_F16 frames: copy the 16-bit samples as they are (no scale, no background)
};

// Batched preparation: the statistics, padded-copy and coverage kernels of
// up to kPrepMax plans in one launch each.  A plan's fixed arguments sit in a
// device table; the frames, their dtype and scales (which change with every
// run) travel in the launch arguments.  off holds three prefix arrays of
// np + 1 ints: workgroups of the statistics, padded-copy and coverage grids.
constexpr int kPrepMax = 64;
// velocity list of the exact recomputation: [0] velocities listed, [1]
// taken, [2] workgroups finished (first job of a launch), [3] unused; then
// the list
constexpr int kFlagHead = 4;
struct PrepJob {
    double* part;
    int nchunk;
    long long npx;
    double* b;
    double* s2;
    float* b32;
    double* P;
    double* Pb;
    PrepArgs pa;  // frames, dtype and scale set per run
    int prep_bx;  // workgroups per frame of the padded copy
    const int* DX;
    const int* DY;
    int ldx, ldy, nvx, nvy, w, h;
    int* IX;
    int* IY;
};
struct PrepBatch {
    const PrepJob* jobs;
    const int* off;
    int np;
    int dtype[kPrepMax];
    const void* frames[kPrepMax];
    const float* scale[kPrepMax];
};
// The merges of up to kPrepMax plans of one stacking round (off: np + 1
// prefix of their velocity counts).
struct MergeJob {
    const int32_t* tcount;
    const Entry* ent;
    int nslot, kt, k_max, nvx, w, k_first;
    // exact recomputation of the velocities whose kept entries may miss one
    // of the k_max best: the launch's arguments (device copy), the list of
    // such velocities (kFlagHead counters, then the velocity indices), and
    // the block shape (x velocities per block, ints per frame record)
    const StackArgs* args;
    int* flag;
    int vbx, rec;
};
struct MergeBatch {
    const MergeJob* jobs;
    const int* off;
    int np;
    sst_candidate* cand[kPrepMax];
    int32_t* count[kPrepMax];
};

// launch wrappers (sst_kernels.hip); each returns a hipError_t
hipError_t launch_stats(const void* frames, int dtype, const float* scale, int n, int h, int w,
                        double* part, int nchunk, double* b, double* s2, float* b32, double* P,
                        double* Pb, double* stats_dev, hipStream_t s);
hipError_t launch_quantize(const float* frames, int n, int h, int w, int dtype, const float* offset,
                           float* part, int nchunk, float* scale, void* q, hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
hipError_t launch_cov(const int* D, int ld, int n, int nv, int size, int* I, hipStream_t s);
hipError_t launch_stack(const StackArgs& a, bool detect, bool staged, int shape, hipStream_t s);
// the frame scales into the records of every velocity block (ord: nblk
// blocks of ord_stride ints, n + kRecPad records of rec ints each)
hipError_t launch_rec_scale(int* ord, int nblk, long long ord_stride, int nrec, int rec, const float* scale,
                            hipStream_t s);
hipError_t launch_stack_batch(const BatchArgs& b, int groups, int shape, hipStream_t s);
// blocks: workgroups of the statistics, padded-copy and coverage grids
hipError_t launch_prep_batch(const PrepBatch& b, const int* blocks, hipStream_t s);
hipError_t launch_merge_batch(const MergeBatch& b, int blocks, hipStream_t s);
hipError_t launch_zero_i32(int* p, int count, hipStream_t s);
hipError_t launch_merge(const int32_t* tcount, const Entry* ent, int nslot, int kt, int k_max,
                        int nvx, int w, int k_first, int nk, void* cand, int32_t* count, int* flag,
                        hipStream_t s);
// Exact lists of the velocities a merge listed (groups workgroups, each
// taking listed velocities until none is left; the last one to finish
// clears the list for the next run).  The single-plan form takes the launch
// arguments by value, the batched form from the jobs.
hipError_t launch_fixup(const StackArgs& a, const MergeJob& job, void* cand, int32_t* count, int groups,
                        hipStream_t s);
hipError_t launch_fixup_batch(const MergeBatch& b, int groups, hipStream_t s);

// The body of sst_detect on a given workspace (sst_api.cpp), shared with
// the entry point that uses the library's static scratch (sst_noalloc.hip),
// and the error-message setter of the C ABI.
int detect_call(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t,
                double t_ref, const double* vx, int nvx, const double* vy, int nvy, float threshold,
                int min_coverage, int k_max, sst_candidate* cand, int32_t* count, double* frame_stats, void* ws,
                size_t ws_bytes, void* stream, bool pinned_upload);
int set_error(int code, const char* msg);

// sub-pixel refinement (sst_refine.hip)
struct RefineArgs {
    const void* frames;  // [n][h][w] of dtype
    int dtype;
    const float* scale;  // [n] for 16-bit frames
    const float* b32;    // [n] frame means (float32)
    const double* P;     // [n+1] variance prefix; P[n] = total variance
    const float* dt;     // [n] t_i - t_ref
    int n, h, w;
    float* params;  // [nc][4] x0, y0, vx, vy (in/out)
    float* snr;     // [nc]
    float* grad;    // [nc][4] or nullptr
    int nc, cutout, steps;
    float lr, inv2s2;  // ascent step; 1 / (2 s^2) of the PSF
    double sw2;        // sum of the squared PSF weights
};
hipError_t launch_refine(const RefineArgs& a, hipStream_t s);

// preprocessing kernels (sst_prep.hip)
constexpr int kMedianMaxFrames = 256;  // frames staged in LDS per pixel column
hipError_t launch_median_sub(const float* F, int n, int h, int w, float* out, float* med, hipStream_t s);
hipError_t launch_coadd(const float* F, int h, int w, int group, int ng, float* out, hipStream_t s);
hipError_t launch_bin2x2(const float* F, int n, int h, int w, float* out, hipStream_t s);

}  // namespace sst
