// HIP kernels of the shift-and-stack search, written for gfx950 (CDNA4):
// wave64, LDS-staged frame tiles, FP32 accumulation, FP64 only for the
// per-frame variance sums of the S/N normaliser.
//
// Data flow of one detect call (paper Sec. 2.1: remove the static sky, shift
// each frame along a trial linear motion, sum, keep significant peaks):
//   k_stats_partial/k_stats_final  per-frame mean b_i, variance s2_i, prefix P
//   k_prep                         zero-padded copy of F_i - b_i (float32);
//                                  16-bit frames are scaled to float32 here
//   k_cov                          per (velocity component, coordinate) the
//                                  first/last frame whose sample is in frame
//   k_stack<detect>                accumulate, S/N, 8-neighbour peaks, keep the
//                                  best kt per (tile, velocity)
//   k_merge                        per-velocity top-k_max, deterministic order
#include "sst_internal.h"
#include "../../include/sst.h"

#include <climits>
#include <cmath>
#include <type_traits>
#include <utility>

namespace sst {

constexpr int kAux = kStatThreads;  // threads of the auxiliary kernels (4 waves)

// ------------------------------------------------------------------ helpers
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that each XCD runs a contiguous range of logical
// work items: neighbouring velocity blocks of one tile then share that XCD's
// L2 copy of the frame region.
__device__ __forceinline__ int xcd_remap(int g, int G) {
    const int per = G / 8, rem = G % 8;
    const int xcd = g % 8, idx = g / 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ double block_sum_f64(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);  // fixed order: deterministic
    __syncthreads();
    return t;
}

__device__ __forceinline__ long long block_sum_i64(long long v, long long* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const long long t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane) {
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    return inc - v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}

// Total order of candidates of one velocity: larger S/N first, then lower
// raster index.  The float is mapped to an unsigned integer with the same
// order; raster indices are distinct, so keys are distinct.
__device__ __forceinline__ unsigned long long cand_key(float sn, int raster) {
    unsigned u = __float_as_uint(sn);
    u ^= (u & 0x80000000u) ? 0xFFFFFFFFu : 0x80000000u;
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)raster);
}

__device__ __forceinline__ i4 load_i4(const int* p) { return *reinterpret_cast<const i4*>(p); }

__device__ __forceinline__ int pick4(const i4 v, int q) {
    return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

// (first, last) frame pair of a coverage interval
__device__ __forceinline__ void load_iv(const int* I, long long e, int& lo, int& hi) {
    const long long v = *reinterpret_cast<const long long*>(I + 2 * e);
    lo = (int)(unsigned)(v & 0xFFFFFFFFll);
    hi = (int)(v >> 32);
}

// ------------------------------------------------------- frame statistics
// One workgroup per (chunk of kStatChunk pixels, frame): the chunk's sum and
// sum of squared deviations from the chunk mean, both float64.
template <int DT>
__device__ __forceinline__ void stats_partial(const void* __restrict__ frames, const float* __restrict__ scale,
                                              long long npx, int nchunk, double* __restrict__ part, int i, int c) {
    const long long f0 = (long long)i * npx;
    const float sc = DT == SST_F32 ? 1.f : scale[i];
    const long long base = (long long)c * kStatChunk;
    const int cnt = (int)min((long long)kStatChunk, npx - base);
    constexpr int PER = kStatChunk / kAux;
    __shared__ double sh[4];
    float v[PER];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = j * kAux + threadIdx.x;
        v[j] = e < cnt ? frame_value<DT>(frames, f0 + base + e, sc) : 0.f;
        s += (double)v[j];
    }
    const double sum = block_sum_f64(s, sh);
    const double mean = sum / (double)cnt;
    double m2 = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = j * kAux + threadIdx.x;
        if (e < cnt) {
            const double d = (double)v[j] - mean;
            m2 += d * d;
        }
    }
    const double M2 = block_sum_f64(m2, sh);
    if (threadIdx.x == 0) {
        double* o = part + ((long long)i * nchunk + c) * 3;
        o[0] = (double)cnt;
        o[1] = sum;
        o[2] = M2;
    }
}

template <int DT>
__global__ __launch_bounds__(kAux) void k_stats_partial(const void* __restrict__ frames,
                                                           const float* __restrict__ scale, long long npx,
                                                           int nchunk, double* __restrict__ part) {
    stats_partial<DT>(frames, scale, npx, nchunk, part, blockIdx.y, blockIdx.x);
}

// Combine the chunks of each frame (pairwise-update formula for the sum of
// squared deviations: M2 = sum_c [M2_c + n_c (mean_c - mean)^2]) and build the
// prefix P[j] = sum_{i<j} s2_i used to normalise any contiguous frame range.
__device__ __forceinline__ void stats_final(const double* __restrict__ part, int nchunk, int n, long long npx,
                                            double* __restrict__ b, double* __restrict__ s2,
                                            float* __restrict__ b32, double* __restrict__ P,
                                            double* __restrict__ Pb, double* __restrict__ stats_dev) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double* p = part + (long long)i * nchunk * 3;
        double sum = 0.0;
        for (int c = 0; c < nchunk; ++c) sum += p[c * 3 + 1];
        const double mean = sum / (double)npx;
        double M2 = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            const double cnt = p[c * 3 + 0];
            const double d = p[c * 3 + 1] / cnt - mean;
            M2 += p[c * 3 + 2] + cnt * d * d;
        }
        const double var = M2 / (double)npx;
        b[i] = mean;
        s2[i] = var;
        b32[i] = (float)mean;
        if (stats_dev) {
            stats_dev[2 * i] = mean;
            stats_dev[2 * i + 1] = var;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        P[0] = 0.0;
        for (int i = 0; i < n; ++i) {
            acc += s2[i];
            P[i + 1] = acc;
        }
    } else if (threadIdx.x == kWave && Pb) {
        // (another wave) the prefix of the means, for searches that subtract
        // the backgrounds after the sum
        double acc = 0.0;
        Pb[0] = 0.0;
        for (int i = 0; i < n; ++i) {
            acc += b[i];
            Pb[i + 1] = acc;
        }
    }
}

__global__ __launch_bounds__(kAux) void k_stats_final(const double* __restrict__ part, int nchunk, int n,
                                                         long long npx, double* __restrict__ b,
                                                         double* __restrict__ s2, float* __restrict__ b32,
                                                         double* __restrict__ P, double* __restrict__ Pb,
                                                         double* __restrict__ stats_dev) {
    stats_final(part, nchunk, n, npx, b, s2, b32, P, Pb, stats_dev);
}

// ------------------------------------------------------------ padded copy
// pad[i] = F_i(x - padL, y - padT) - b32[i] inside the frame, 0 outside, in
// row groups: element (y, x) at float ((y / 4) * Wp + x) * 4 + y % 4.  Out-of-
// frame samples then add nothing, and the stack kernel stages any window
// with unconditional 16-byte loads, each holding four rows of one column.
// One thread per 16-byte chunk (row group, column) of a frame; consecutive
// threads take consecutive columns, so the four row reads and the chunk
// write are coalesced.
// The 16-bit copy (IEEE half samples as stored, zero outside): the same
// layout with 8-byte chunks, frame i at half index 2 i Hp Wp.
__global__ __launch_bounds__(kAux) void k_prep_half(const PrepArgs a) {
    const int i = blockIdx.y;
    const unsigned q = blockIdx.x * kAux + threadIdx.x;
    const unsigned ng = (unsigned)a.Hp / 4;
    if (q >= ng * (unsigned)a.Wp) return;
    const int g = (int)(q / (unsigned)a.Wp);
    const int xp = (int)(q - (unsigned)g * (unsigned)a.Wp);
    const int x = xp - a.padL;
    unsigned o[4] = {0u, 0u, 0u, 0u};
    if (x >= 0 && x < a.w) {
        const uint16_t* f = static_cast<const uint16_t*>(a.frames);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int y = 4 * g + k - a.padT;
            if (y >= 0 && y < a.h) o[k] = f[((long long)i * a.h + y) * a.w + x];
        }
    }
    typedef unsigned u2v __attribute__((ext_vector_type(2)));
    u2v* dst = reinterpret_cast<u2v*>(reinterpret_cast<uint16_t*>(a.pad) + 2 * (long long)i * a.Hp * a.Wp +
                                      (long long)q * 4);
    *dst = u2v{o[0] | (o[1] << 16), o[2] | (o[3] << 16)};
}

template <int DT>
__device__ __forceinline__ void prep(const PrepArgs& a, int i, int bx) {
    // (a padded frame has fewer than 2^31 bytes on the staged path and far
    // fewer than 2^32 chunks on any path: sides are at most about 3 x 16384)
    const unsigned q = bx * kAux + threadIdx.x;
    const unsigned ng = (unsigned)a.Hp / 4;
    if (q >= ng * (unsigned)a.Wp) return;
    const int g = (int)(q / (unsigned)a.Wp);
    const int xp = (int)(q - (unsigned)g * (unsigned)a.Wp);
    const int x = xp - a.padL;
    float o[4] = {0.f, 0.f, 0.f, 0.f};
    if (x >= 0 && x < a.w) {
        const float bb = a.b32 ? a.b32[i] : 0.f;
        const float sc = DT == SST_F32 ? 1.f : a.scale[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int y = 4 * g + k - a.padT;
            if (y >= 0 && y < a.h) o[k] = frame_value<DT>(a.frames, ((long long)i * a.h + y) * a.w + x, sc) - bb;
        }
    }
    f4* dst = reinterpret_cast<f4*>(a.pad + (long long)i * a.Hp * a.Wp + (long long)q * 4);
    *dst = f4{o[0], o[1], o[2], o[3]};
}

template <int DT>
__global__ __launch_bounds__(kAux) void k_prep(const PrepArgs a) {
    prep<DT>(a, blockIdx.y, blockIdx.x);
}

// -------------------------------------------------------------- quantiser
// 16-bit storage with a per-frame offset o_i (0, or float32 of the frame
// mean) and scale s_i = max|F_i - o_i| * 2^-14 (1 for a constant frame):
// stored q = round-to-nearest-even of the float32 quotient (F - o_i) / s_i
// (the difference rounded to float32 first) in bfloat16 or IEEE half.
// |q| <= 2^14, so neither format overflows.
__global__ __launch_bounds__(kAux) void k_absmax_partial(const float* __restrict__ frames, long long npx,
                                                            const float* __restrict__ offset, int nchunk,
                                                            float* __restrict__ part) {
    const int i = blockIdx.y, c = blockIdx.x;
    const float* f = frames + (long long)i * npx;
    const float off = offset ? offset[i] : 0.f;
    const long long base = (long long)c * kStatChunk;
    const int cnt = (int)min((long long)kStatChunk, npx - base);
    float m = 0.f;
    for (int e = threadIdx.x; e < cnt; e += kAux) m = fmaxf(m, fabsf(f[base + e] - off));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)i * nchunk + c] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__global__ __launch_bounds__(kAux) void k_absmax_final(const float* __restrict__ part, int nchunk, int n,
                                                          float* __restrict__ scale) {
    for (int i = threadIdx.x; i < n; i += kAux) {
        float m = 0.f;
        for (int c = 0; c < nchunk; ++c) m = fmaxf(m, part[(long long)i * nchunk + c]);
        scale[i] = m > 0.f ? ldexpf(m, -14) : 1.f;
    }
}

// float32 -> bfloat16 bits, round to nearest even (finite input)
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int DT>
__global__ __launch_bounds__(kAux) void k_quantize(const float* __restrict__ frames, long long npx,
                                                      const float* __restrict__ offset,
                                                      const float* __restrict__ scale, uint16_t* __restrict__ q) {
    const int i = blockIdx.y;
    const long long e = (long long)blockIdx.x * kAux + threadIdx.x;
    if (e >= npx) return;
    const float off = offset ? offset[i] : 0.f;
    const float v = (frames[(long long)i * npx + e] - off) / scale[i];
    uint16_t bits;
    if constexpr (DT == SST_BF16) {
        bits = bf16_rne(v);
    } else {
        bits = __builtin_bit_cast(uint16_t, (_Float16)v);
    }
    q[(long long)i * npx + e] = bits;
}

// ------------------------------------------------------ coverage intervals
// I[a][x] = (first, last) frame i with 0 <= x + D[i][a] < size.  D is
// monotone in i (the timestamps are sorted), so the in-frame frames form one
// interval and the 2-D coverage of a pixel is the intersection of its x and
// y intervals.  Empty: (n, -1).
__device__ __forceinline__ void cov(const int* __restrict__ D, int ld, int n, int size, int* __restrict__ I,
                                    int a, int bx) {
    const int x = bx * kAux + threadIdx.x;
    if (x >= size) return;
    int lo = n, hi = -1;
    for (int i = 0; i < n; ++i) {
        const int p = x + D[(long long)i * ld + a];
        if (p >= 0 && p < size) {
            lo = min(lo, i);
            hi = i;
        }
    }
    I[2 * ((long long)a * size + x)] = lo;
    I[2 * ((long long)a * size + x) + 1] = hi;
}

__global__ __launch_bounds__(kAux) void k_cov(const int* __restrict__ D, int ld, int n, int size,
                                                 int* __restrict__ I) {
    cov(D, ld, n, size, I, blockIdx.y, blockIdx.x);
}

__device__ __forceinline__ int coverage(int xlo, int xhi, int ylo, int yhi, int& lo, int& hi) {
    lo = max(xlo, ylo);
    hi = min(xhi, yhi);
    return hi - lo + 1;
}

// -------------------------------------------------------------- stacking
// A work item is a tile (64 columns x 32 rows) and a velocity block (VBX x
// velocities, one pair of y velocities).  Per frame the workgroup stages one
// window of the padded copy into LDS: kRG row groups by CW columns starting
// at the tile origin shifted by the block's smallest x shift and by the
// smaller of the pair's y shifts, rounded down to a row group.  Every
// velocity of the block then reads its samples from that window: lane l of
// x velocity a reads column c_a + l, y velocity b reads rows from f_b, with
// one 16-byte LDS read per four rows.  The row phases (f0, f1) of a frame
// select one of kNCase read patterns; the host sorts each block's frames by
// pattern and the kernel runs one loop per pattern, so every read and add is
// fixed at compile time and no per-frame dispatch remains.  Frames are summed
// in that order (the float32 sum of the same terms, in a fixed order that
// depends only on the block and the frames' shifts).
//
// Staging is a ring of NBUF buffers: while frame k is added, frames k + 1 ..
// k + NBUF - 2 have been issued and frame k + NBUF - 1 is issued now; each
// wave waits only for its own loads of frame k + 1 before the barrier that
// ends frame k.  Loads go straight to LDS (buffer load with LDS destination:
// lane l's 16 bytes land at the instruction's base + 16 l), each frame through
// its own buffer descriptor (the frame's padded copy is below 2^31 bytes on
// this path).  The workgroup has exactly one LDS object: with several, the
// compiler makes every LDS read wait for all pending LDS-destination loads.

typedef const __attribute__((address_space(3))) int LInt;
typedef const __attribute__((address_space(3))) float LFloat;
// read-only tables of the launch (the frame order): uniform loads are scalar
typedef const __attribute__((address_space(4))) int CInt;

// float index of element (y, x) of a padded frame in row-group layout
__device__ __forceinline__ long long pad_at(int y, int x, int Wp) {
    return ((long long)(y >> 2) * Wp + x) * 4 + (y & 3);
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Read pattern C: row phases f0, f1 of the pair's first rows in the groups
// read, and the number of row groups holding a wave's 16 rows from a phase.
template <int C>
struct Case {
    static constexpr bool shared = C < kNShared;
    static constexpr int lo = C / 9, dd = C % 9 - 4;
    static constexpr int f0 = shared ? (dd >= 0 ? lo : lo - dd) : (C - kNShared) / 4;
    static constexpr int f1 = shared ? (dd >= 0 ? lo + dd : lo) : (C - kNShared) % 4;
    static constexpr int g0 = (f0 + kRowsW - 1) / 4 + 1;
    static constexpr int g1 = (f1 + kRowsW - 1) / 4 + 1;
    static constexpr int gs = (cmax(f0, f1) + kRowsW - 1) / 4 + 1;
    // the lower row half of a whole tile reads from row group 4 of the
    // window on (a split item's window starts at its half); a separate read
    // may start up to shape_max_sep groups further (the host checks that)
    static_assert(!shared || 4 + gs <= kRG, "a shared read stays inside the window");
    static_assert(!shared || gs <= 6, "a shared read stays inside a split item's window");
    static_assert(shared || 4 + cmax(g0, g1) <= 9, "separate reads span at most 5 row groups");
};

// four rows of one column: float32 samples, or 16-bit samples (row k of the
// group in half k % 2 of dword k / 2)
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// G row groups of one column from p (group stride CW chunks) into v
template <int G, int CW, typename T>
__device__ __forceinline__ void read_groups(const T* p, T (&v)[6]) {
    static_assert(G <= 6, "at most 24 rows");
#pragma unroll
    for (int j = 0; j < G; ++j) v[j] = p[j * CW];
}

// a[r] += sample r + F of the read (float32), or a[r] = fma(sample, sc,
// a[r]) (16-bit: the sample widened exactly, times the frame's scale, added
// with one rounding)
template <int F>
__device__ __forceinline__ void add_rows(const f4 (&v)[6], float, float (&a)[kRowsW]) {
    static_assert(F + kRowsW <= 24, "rows inside the read");
#pragma unroll
    for (int r = 0; r < kRowsW; ++r) a[r] += v[(r + F) / 4][(r + F) % 4];
}

template <int F>
__device__ __forceinline__ void add_rows(const u2 (&v)[6], float sc, float (&a)[kRowsW]) {
    static_assert(F + kRowsW <= 24, "rows inside the read");
#pragma unroll
    for (int r = 0; r < kRowsW; ++r) {
        const int k = r + F;
        // (the dword selected into a scalar first: a bit_cast of a vector
        // element expression reads element 0)
        const unsigned d = ((k % 4) / 2) ? v[k / 4].y : v[k / 4].x;
        const h2 pr = __builtin_bit_cast(h2, d);
        const float x = (k % 2) ? (float)pr.y : (float)pr.x;
        a[r] = __builtin_fmaf(x, sc, a[r]);
    }
}

// Keeps the G groups of v live up to this point: a group's components that
// no add uses would otherwise count as dead at once, and their registers be
// handed to the next read while the load into them is still in flight
// (costing a wait for every LDS read outstanding).
template <int G, typename T>
__device__ __forceinline__ void hold(const T (&v)[6]) {
#pragma unroll
    for (int j = 0; j < G; ++j) asm volatile("" ::"v"(v[j]));
}

// Frame k's adds for the wave's kVPW x velocities (columns col[q]) in
// pattern C; base = the wave's first row group of the staged window at lane
// column 0; go0, go1 = row-group offsets of the two y velocities (separate
// patterns only).  The reads of the next x velocity are issued before the
// adds of the current one.
template <int C, int CW, typename T>
__device__ __forceinline__ void add_frame(const T* base, const int (&col)[kVPW], int go0, int go1, float sc,
                                          float (&acc)[kVPW][kVYW][kRowsW]) {
    using K = Case<C>;
    static_assert(kVPW == 3, "three x velocities per wave");
    T va[6], vb[6];
    if constexpr (K::shared) {
        constexpr int G = K::gs;
        read_groups<G, CW>(base + col[0], va);
        read_groups<G, CW>(base + col[1], vb);
        add_rows<K::f0>(va, sc, acc[0][0]);
        add_rows<K::f1>(va, sc, acc[0][1]);
        hold<G>(va);
        read_groups<G, CW>(base + col[2], va);
        add_rows<K::f0>(vb, sc, acc[1][0]);
        add_rows<K::f1>(vb, sc, acc[1][1]);
        hold<G>(vb);
        add_rows<K::f0>(va, sc, acc[2][0]);
        add_rows<K::f1>(va, sc, acc[2][1]);
        hold<G>(va);
    } else {
        const T* b0 = base + go0 * CW;
        const T* b1 = base + go1 * CW;
#pragma unroll
        for (int q = 0; q < kVPW; ++q) {
            read_groups<K::g0, CW>(b0 + col[q], va);
            read_groups<K::g1, CW>(b1 + col[q], vb);
            add_rows<K::f0>(va, sc, acc[q][0]);
            hold<K::g0>(va);
            add_rows<K::f1>(vb, sc, acc[q][1]);
            hold<K::g1>(vb);
        }
    }
}

// add_frame with one read in flight at a time: fewer registers (the plain
// stack of shape 2, at four waves per SIMD)
template <int C, int CW, typename T>
__device__ __forceinline__ void add_frame1(const T* base, const int (&col)[kVPW], int go0, int go1, float sc,
                                           float (&acc)[kVPW][kVYW][kRowsW]) {
    using K = Case<C>;
    T va[6], vb[6];
    if constexpr (K::shared) {
        constexpr int G = K::gs;
#pragma unroll
        for (int q = 0; q < kVPW; ++q) {
            read_groups<G, CW>(base + col[q], va);
            add_rows<K::f0>(va, sc, acc[q][0]);
            add_rows<K::f1>(va, sc, acc[q][1]);
            hold<G>(va);
        }
    } else {
        const T* b0 = base + go0 * CW;
        const T* b1 = base + go1 * CW;
#pragma unroll
        for (int q = 0; q < kVPW; ++q) {
            read_groups<K::g0, CW>(b0 + col[q], va);
            add_rows<K::f0>(va, sc, acc[q][0]);
            hold<K::g0>(va);
            read_groups<K::g1, CW>(b1 + col[q], vb);
            add_rows<K::f1>(vb, sc, acc[q][1]);
            hold<K::g1>(vb);
        }
    }
}

// This wave's share of one frame's staging: its loads j < nst (instruction
// wave + NW j of the frame), each 64 lanes x 16 bytes from the padded frame
// at byte offsets voff[j] + soff into buf + 64 (wave + NW j) chunks.
template <int NW, int NSTX>
__device__ __forceinline__ void stage_window(const float* frame, int fbytes, const int (&voff)[NSTX], int nst,
                                             int soff, float* buf, int wave) {
    // (device pass only: the host pass of a template instantiated from a
    // lambda cannot resolve the buffer-resource builtins)
#if defined(__HIP_DEVICE_COMPILE__)
    const auto rs = __builtin_amdgcn_make_buffer_rsrc((void*)frame, 0, fbytes, 0x00020000);
#pragma unroll
    for (int j = 0; j < NSTX; ++j) {
        if (j < nst) {
            auto* dst = (__attribute__((address_space(3))) void*)(buf + (wave + NW * j) * kWave * 4);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 16, voff[j], soff, 0, 0);
        }
    }
#endif
}

// Wait until at most N of this wave's loads into LDS are in flight (vmcnt N;
// expcnt and lgkmcnt not waited for).
template <int N>
__device__ __forceinline__ void wait_loads() {
    static_assert(N >= 0 && N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// Workgroup barrier with no memory fence: every wave has already waited for
// its own loads into LDS, and a staging buffer is refilled only after the
// barrier that follows the last reads of its frame.  (A fenced barrier would
// make each wave wait for all of its loads, including the frames still
// meant to be in flight.)
__device__ __forceinline__ void barrier_no_fence() { asm volatile("s_barrier" ::: "memory"); }

// S/N, peak test and candidate output of one (tile, velocity) for one wave.
// Tiles do not overlap: the wave holds rows 16h .. 16h + 15 (h = row half)
// of the tile, one column per lane, and may emit any of them.  The peak test
// of the wave's rows next to the other half needs that half's boundary row,
// which every wave publishes in LDS after the frame loop.  The candidate
// search works on a column of kColRows rows, tile rows R0 .. R0 + 17 with
// R0 = 16h - 1: the wave's own 16 rows (column rows 1 .. 16), the other
// half's boundary row and, on the tile's outer side, the row of the next
// tile, which this workgroup does not hold.  Neighbours outside the tile
// (that row, and the columns left of lane 0 and right of lane 63) first
// count as -infinity; a pixel that passes the test against everything
// inside the tile then has its outside neighbours' S/N evaluated directly,
// a sum over the frames of the padded copy in the block's frame order: the
// same float32 adds of the same values as the workgroup that owns that
// pixel, hence the same S/N.  The S/N of a row is recomputed where it is
// needed rather than stored, to keep the register footprint of this
// epilogue below the main loop's.
constexpr int kColRows = kRowsW + 2;
constexpr unsigned kEmitRows = ((1u << (kColRows - 1)) - 1u) & ~1u;  // column rows 1 .. kColRows - 2

struct SnCtx {
    LInt* IYr;    // [kColRows][2] y coverage intervals of the column's rows
    LFloat* RSr;  // [kColRows] 1/sqrt(V) of a pixel whose x samples are all inside
    const double* P;   // prefix sums of the frame variances
    int n, xlo, xhi;
    bool xfull;        // this lane's column sees every frame in x
};

// Where a callee reads the arguments of the work item: the kernel argument
// segment, or the entry of a batch's argument table (never a copy).
typedef const StackArgs* KArgs;

// S/N of column row r of this lane (and its coverage).  A lane whose x
// samples are all inside has coverage = the row's y interval, whose 1/sqrt(V)
// is tabulated per row; other lanes combine both intervals.  Both forms are
// the same arithmetic, rsqrtf((float)(P[hi + 1] - P[lo])) times the sum.
__device__ __forceinline__ float sn_row(const SnCtx& c, float acc, int r, int& cov) {
    const int ylo = c.IYr[2 * r], yhi = c.IYr[2 * r + 1];
    if (c.xfull) {
        cov = yhi - ylo + 1;
        return cov > 0 ? acc * c.RSr[r] : -INFINITY;
    }
    int lo, hi;
    cov = coverage(c.xlo, c.xhi, ylo, yhi, lo, hi);
    if (cov <= 0) return -INFINITY;
    const double V = c.P[hi + 1] - c.P[lo];
    return V > 0.0 ? acc * rsqrtf((float)V) : 0.f;
}

// S/N of pixel (x, y) at velocity (a, b) evaluated on its own: the sum of its
// shifted samples of the padded copy in its block's frame order (the order of
// the work items), then the same normalisation as sn_row.  vbx and rec are
// the shape's block width and record size.
__device__ __forceinline__ float sn_direct(KArgs A, const double* P, int a, int b, int x, int y, int vbx, int rec) {
    if (x < 0 || x >= A->w || y < 0 || y >= A->h) return -INFINITY;
    int xlo, xhi, ylo, yhi, lo, hi;
    load_iv(A->IX, (long long)a * A->w + x, xlo, xhi);
    load_iv(A->IY, (long long)b * A->h + y, ylo, yhi);
    if (coverage(xlo, xhi, ylo, yhi, lo, hi) <= 0) return -INFINITY;
    typedef const __attribute__((address_space(1))) float GFloat;
    typedef const __attribute__((address_space(1))) int GInt;
    GFloat* pad = (GFloat*)A->pad;
    GInt* DX = (GInt*)A->DX;
    GInt* DY = (GInt*)A->DY;
    GInt* ordr = (GInt*)(A->ord + (long long)((b / kVYW) * A->nvbx + a / vbx) * A->ord_stride + kCountInts);
    const long long fstride = A->fstride;
    const int Wp = A->Wp, ldx = A->ldx, ldy = A->ldy, n = A->n;
    const int x0 = x + A->padL, y0 = y + A->padT;
    float acc = 0.f;
    if (A->half) {
        // 16-bit copy: fma of each sample with its frame's scale, then the
        // backgrounds of the covering frames (the stacking loop's arithmetic)
        typedef const __attribute__((address_space(1))) _Float16 GHalf;
        typedef const __attribute__((address_space(1))) double GDouble;
        GHalf* pad16 = (GHalf*)A->pad;
        GFloat* sc = (GFloat*)A->scale;
#pragma unroll 1
        for (int k = 0; k < n; ++k) {
            const int i = ordr[(long long)k * rec + 4];
            const int dx = DX[(long long)i * ldx + a], dy = DY[(long long)i * ldy + b];
            const float v = (float)pad16[2 * (long long)i * fstride + pad_at(y0 + dy, x0 + dx, Wp)];
            acc = __builtin_fmaf(v, sc[i], acc);
        }
        GDouble* Pb = (GDouble*)A->Pb;
        acc -= (float)(Pb[hi + 1] - Pb[lo]);
    } else {
#pragma unroll 1
        for (int k = 0; k < n; ++k) {
            const int i = ordr[(long long)k * rec + 4];
            const int dx = DX[(long long)i * ldx + a], dy = DY[(long long)i * ldy + b];
            acc += pad[(long long)i * fstride + pad_at(y0 + dy, x0 + dx, Wp)];
        }
    }
    const double V = P[hi + 1] - P[lo];
    return V > 0.0 ? acc * rsqrtf((float)V) : 0.f;
}

// Peak test and candidate output for one (tile, velocity, row half) whose
// column sums are parked in LDS: col[r * 64 + lane] = S' of column row r.
// fl marks the rows (1 .. kColRows - 2) that pass threshold and coverage;
// orow is the column row outside the tile (0 or kColRows - 1); for an item
// of one row half (SPLIT) both rows 0 and kColRows - 1 lie outside it.  The
// (tile, velocity, row half) writes its count and kept entries to slot.
template <bool SPLIT>
__device__ __noinline__ void candidates_from_column(KArgs A, LInt* IYr, LFloat* RSr, const double* P,
                                                    int xlo, int xhi, int a, int b, long long slot,
                                                    LFloat* col, unsigned fl, int lane, int x, int Yc,
                                                    int orow, int vbx, int rec) {
    auto outside_row = [&](int r) __attribute__((always_inline)) {
        return SPLIT ? (r == 0 || r == kColRows - 1) : r == orow;
    };
    SnCtx c;
    c.IYr = IYr;
    c.RSr = RSr;
    c.P = P;
    c.n = A->n;
    c.xlo = xlo;
    c.xhi = xhi;
    c.xfull = xlo == 0 && xhi == c.n - 1;
    const int kt = A->kt, w = A->w;
    // 8-neighbour test with the raster tie rule: neighbours earlier in raster
    // order must be strictly smaller, later ones may tie.  Outside the tile:
    // -infinity for now.
    auto sn_col = [&](int r) __attribute__((always_inline)) {
        int cv;
        return outside_row(r) ? -INFINITY : sn_row(c, col[r * kWave + lane], r, cv);
    };
    // the left and right neighbours' values by whole-wave DPP shifts (lane 0
    // and lane 63 have none: -infinity)
    auto left = [&](float v) __attribute__((always_inline)) {
        return __int_as_float(
            __builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(v), 0x138, 0xf, 0xf, false));
    };
    auto right = [&](float v) __attribute__((always_inline)) {
        return __int_as_float(
            __builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(v), 0x130, 0xf, 0xf, false));
    };
    unsigned cm = 0;
    float Sm = sn_col(0), S0 = sn_col(1);
    float Lm = left(Sm), Rm = right(Sm);
    float L0 = left(S0), R0 = right(S0);
    // (unrolled: the LDS reads of later rows are issued early)
#pragma unroll
    for (int r = 1; r <= kColRows - 2; ++r) {
        const float Sp = sn_col(r + 1);
        const float Lp = left(Sp), Rp = right(Sp);
        if ((fl >> r) & 1u) {
            const float s = S0;
            const bool ok = s > Lm && s > Sm && s > Rm && s > L0 && s >= R0 && s >= Lp && s >= Sp && s >= Rp;
            if (ok) cm |= 1u << r;
        }
        Sm = S0;
        S0 = Sp;
        Lm = L0;
        Rm = R0;
        L0 = Lp;
        R0 = Rp;
    }
    // pixels next to the tile's border: test the outside neighbours
    // (own rows next to an outside row)
    const unsigned erows = SPLIT ? (2u | (1u << (kColRows - 2))) : (1u << (orow == 0 ? 1 : kColRows - 2));
    unsigned todo = cm & ((lane == 0 || lane == kWave - 1) ? kEmitRows : erows);
#pragma unroll 1
    while (todo != 0) {
        const int r = __builtin_ctz(todo);
        todo &= todo - 1;
        int cv;
        const float s = sn_row(c, col[r * kWave + lane], r, cv);
        bool ok = true;
#pragma unroll 1
        for (int k = 0; k < 9 && ok; ++k) {
            const int dy = k / 3 - 1, dx = k % 3 - 1;
            const bool outside = lane + dx < 0 || lane + dx >= kWave || outside_row(r + dy);
            if (k == 4 || !outside) continue;
            const float sq = sn_direct(A, P, a, b, x + dx, Yc + r + dy, vbx, rec);
            const bool earlier = dy < 0 || (dy == 0 && dx < 0);
            ok = earlier ? s > sq : s >= sq;
        }
        if (!ok) cm &= ~(1u << r);
    }
    typedef __attribute__((address_space(1))) int32_t GInt;
    const int total = wave_sum_i32(__popc(cm));
    if (lane == 0) ((GInt*)A->tcount)[slot] = total;
    if (total == 0) return;
    Entry* E = A->ent + slot * (long long)kt;
    if (total <= kt) {
        int k = wave_excl_scan(__popc(cm), lane);
#pragma unroll 1
        for (int r = 1; r <= kColRows - 2; ++r) {
            if ((cm >> r) & 1u) {
                int cov;
                const float v = col[r * kWave + lane];
                const float s = sn_row(c, v, r, cov);
                E[k++] = Entry{s, v, (Yc + r) * w + x, cov};
            }
        }
        return;
    }
    // more candidates than kept entries: keep the kt best keys
    unsigned left_rows = cm;
#pragma unroll 1
    for (int k = 0; k < kt; ++k) {
        unsigned long long best = 0;
        int bestr = -1;
#pragma unroll 1
        for (int r = 1; r <= kColRows - 2; ++r) {
            if ((left_rows >> r) & 1u) {
                int cov;
                const unsigned long long key = cand_key(sn_row(c, col[r * kWave + lane], r, cov), (Yc + r) * w + x);
                if (key > best) {
                    best = key;
                    bestr = r;
                }
            }
        }
        const unsigned long long wb = wave_max_u64(best);
        if (bestr >= 0 && best == wb) {
            int cov;
            const float v = col[bestr * kWave + lane];
            E[k] = Entry{sn_row(c, v, bestr, cov), v, (Yc + bestr) * w + x, cov};
            left_rows &= ~(1u << bestr);
        }
    }
}

// rsm[r]: for a lane whose x samples are all inside, 1/sqrt(V) of the wave's
// row r if that row can hold a candidate (inside the grid, coverage >= c_min),
// else NaN, so that acc * rsm[r] > threshold is exactly the threshold and
// coverage test (NaN compares false).  xrow is the other row half's boundary
// row of the same velocity (NULL for an item of one row half, whose both
// boundary rows lie outside it); IYr and RSr start at column row 0 (tile
// row R0).
template <bool SPLIT, bool DEFER>
__device__ __forceinline__ void detect_epilogue(const StackArgs& A, KArgs Ap, const float (&acc)[kRowsW],
                                                const float (&rsm)[kRowsW], int a, int b, int x, bool xin, int lane,
                                                int h, int Y0, int tile, float* col, const float* xrow,
                                                const int* IYr, const float* RSr, const double* P, int xlo, int xhi,
                                                int vbx, int rec, int* sflag) {
    const long long kc = (long long)(b - A.vby0 * kVYW) * A.nvx + a;
    const long long slot = kc * A.nslot + 2 * tile + h;
    SnCtx c;
    c.IYr = (LInt*)IYr;
    c.RSr = (LFloat*)RSr;
    c.P = P;
    c.n = A.n;
    c.xlo = xlo;
    c.xhi = xhi;
    c.xfull = xlo == 0 && xhi == A.n - 1;
    unsigned fl = 0;  // bit r: the wave's row r passes threshold and coverage
    if (c.xfull && xin) {
        // the largest product first (fmaxf skips NaN, so m is one of the
        // rows that can hold a candidate, or NaN); rows only when it passes
        float m = acc[0] * rsm[0];
#pragma unroll
        for (int r = 1; r < kRowsW; ++r) m = fmaxf(m, acc[r] * rsm[r]);
        if (m > A.thr) {
#pragma unroll
            for (int r = 0; r < kRowsW; ++r)
                if (acc[r] * rsm[r] > A.thr) fl |= 1u << r;
        }
    }
    if (__ballot(!c.xfull && xin) != 0) {
        // lanes near the frame's x edges: combine both coverage intervals
        if (!c.xfull && xin) {
            if constexpr (DEFER) {
                // (few registers: each row's multiplier, as sn_row forms
                // the S/N, through this wave's column area, then the rows
                // tested as for inside lanes; NaN where the row cannot hold
                // a candidate)
#pragma unroll 1
                for (int r = 0; r < kRowsW; ++r) {
                    int lo, hi;
                    const int cov = coverage(xlo, xhi, IYr[2 * (r + 1)], IYr[2 * (r + 1) + 1], lo, hi);
                    float m = __builtin_nanf("");
                    if (cov > 0 && cov >= A.cmin) {
                        const double V = P[hi + 1] - P[lo];
                        m = V > 0.0 ? rsqrtf((float)V) : 0.f;
                    }
                    col[r * kWave + lane] = m;
                }
#pragma unroll
                for (int r = 0; r < kRowsW; ++r)
                    if (acc[r] * col[r * kWave + lane] > A.thr) fl |= 1u << r;
            } else {
#pragma unroll
                for (int r = 0; r < kRowsW; ++r) {
                    int cov;
                    const float s = sn_row(c, acc[r], r + 1, cov);
                    if (cov >= A.cmin && s > A.thr) fl |= 1u << r;
                }
            }
        }
    }
    fl <<= 1;  // the wave's row r is column row r + 1
    if (__ballot(fl != 0) == 0) {
        if (lane == 0) A.tcount[slot] = 0;
        return;
    }
    if constexpr (DEFER) {
        // the second pass finds this slot's candidates
        *sflag = 1;
    } else {
        // Rare path (some pixel of this wave's column block clears the
        // threshold): park the sums in this wave's LDS slot and work from
        // there with runtime row loops, which keeps this code's register use
        // small.
        float* own = col + kWave;
#pragma unroll
        for (int r = 0; r < kRowsW; ++r) own[r * kWave + lane] = acc[r];
        if constexpr (!SPLIT) col[(h ? 0 : kColRows - 1) * kWave + lane] = xrow[lane];
        candidates_from_column<SPLIT>(Ap, (LInt*)IYr, (LFloat*)RSr, P, xlo, xhi, a, b, slot, (LFloat*)col, fl, lane, x,
                                      Y0 + kRowsW * h - 1, h ? kColRows - 1 : 0, vbx, rec);
    }
}

template <int V>
using ic = std::integral_constant<int, V>;

// f(ic<C>{}) for every C of the sequence, in order
template <typename F, int... Cs>
__device__ __forceinline__ void for_cases(F& f, std::integer_sequence<int, Cs...>) {
    (f(ic<Cs>{}), ...);
}

// LDS floats of a workgroup of shape SH: the staging ring (float32 windows,
// the larger), or after the frame loop the epilogue's areas (candidate
// columns, exchanged boundary rows, coverage, normaliser and background
// tables, variance prefix), whichever is larger, plus one int for the batch
// kernel's work counter.
template <int SH, int NB>
struct Lds {
    static constexpr int NW = shape_waves(SH);
    static constexpr int buf = shape_ni_max(SH) * kWave * 4;  // floats per staging buffer
    static constexpr int stage = NB * buf;
    static constexpr int colf = NW * kColRows * kWave;
    static constexpr int xch = NW * kVPW * kVYW * kWave;
    static constexpr int iy = ((kVYW * kRows + 1) * 2 + 3) / 4 * 4;  // (areas stay 16-byte aligned)
    static constexpr int rs = (kVYW * kRows + 1 + 3) / 4 * 4;
    static constexpr int rm = kVYW * kRows;
    static constexpr int cb = kVYW * kRows;
    static constexpr int p = 2 * kPLds;  // doubles
    static constexpr int epi = colf + xch + iy + rs + rm + cb + p;
    static constexpr int total = (stage > epi ? stage : epi) + 4;
};

// Staging buffers of the stacking kernels: the one-pass search of shape 2
// waits at a barrier every second frame (four buffers); its first pass of
// two (DEFER) and the plain stack keep the shape's ring and run four
// workgroups per CU.
__host__ __device__ constexpr bool item_pair(int sh, bool detect, bool defer) { return sh == 2 && detect && !defer; }
__host__ __device__ constexpr int item_nbuf(int sh, bool detect, bool defer) {
    return ring_bufs(sh, item_pair(sh, detect, defer));
}
__host__ __device__ constexpr int item_waves_per_eu(int sh, bool detect, bool defer) {
    return sh == 2 && (!detect || defer) ? 4 : 3;
}

// One work item of the stacking kernels: tile and velocity block number
// `logical` of the problem A describes (Ap: where a callee reads A); lds is
// the workgroup's LDS array (Lds<SH, DETECT>::total floats).
// DEFER (first pass of a two-pass search of shape 2): no candidate search;
// an item with a pixel above threshold is marked in A.redo for the second
// pass, which runs it again in full.
template <bool DETECT, bool STAGED, int SH, bool HALF = false, bool DEFER = false>
__device__ __forceinline__ void stack_item(const StackArgs& A, KArgs Ap, int logical, float* lds) {
    static_assert(!DEFER || (DETECT && STAGED && !HALF && SH == 2), "two passes: the float32 search of shape 2");
    static_assert(!HALF || (DETECT && STAGED), "16-bit samples: the staged search only");
    constexpr int NW = shape_waves(SH), VBX = shape_vbx(SH);
    constexpr int CW = HALF ? shape_cw_half(SH) : shape_cw_max(SH);  // window columns
    constexpr int CB = HALF ? 8 : 16;  // bytes of four rows of one column
    // the one-pass search of shape 2 waits at a barrier every second frame
    constexpr bool PAIR = item_pair(SH, DETECT, DEFER);
    constexpr int NBUF = item_nbuf(SH, DETECT, DEFER), REC = shape_rec_ints(SH);
    static_assert(!PAIR || NBUF == 4, "two frames in flight while two are added");
    constexpr int NI = HALF ? shape_ni_half(SH) : shape_ni_max(SH);
    constexpr int BUFF = NI * kWave * 4;      // floats per staging buffer
    static_assert(BUFF <= Lds<SH, NBUF>::buf, "buffers inside the ring");
    constexpr int NSTX = (NI + NW - 1) / NW;  // most staging loads per wave and frame
    using T = typename std::conditional<HALF, u2, f4>::type;
    static_assert(NI >= NW && NSTX * (NBUF - 2 > 0 ? NBUF - 2 : 1) < 16, "every wave stages; vmcnt field");
    static_assert(NBUF <= kRecPad, "records read ahead stay inside the block's list");
    constexpr bool SPLIT = shape_split(SH);  // the item is one row half of the tile
    constexpr int RG = shape_rg(SH);         // row groups of the window
    static_assert(!SPLIT || RG >= 6, "a split item's window holds every shared read");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nvb = A.nvbx * A.nvby;
    // (SPLIT: the two row halves of a (tile, block) are consecutive items)
    const int titem = SPLIT ? logical >> 1 : logical / nvb;
    const int vb = SPLIT ? titem % nvb : logical - titem * nvb;
    const int tile = SPLIT ? titem / nvb : titem;
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int bxi = vb % A.nvbx, byi = A.vby0 + vb / A.nvbx;
    const int a0 = bxi * VBX;
    const int b0 = byi * kVYW;  // the pair's first y velocity
    const int xg = SPLIT ? wave : wave >> 1;  // which kVPW-group of the block's x velocities
    const int h = SPLIT ? (logical & 1) : (wave & 1);  // row half
    const int aw = a0 + kVPW * xg;  // this wave's first x velocity
    const int X0 = tx * kTileW;
    const int Y0 = ty * kRows;
    // waves whose velocities all lie past the grid (in a partial last block)
    // only help stage the frames
    const bool busy = aw < A.nvx && b0 < A.nvy;
    // (DEFER) set by a wave whose rows hold a pixel above threshold; cleared
    // before the first barrier, set after the frame loop
    int* const s_redo = reinterpret_cast<int*>(lds + Lds<SH, NBUF>::total - 4);
    if constexpr (DEFER) {
        // once more than 1 / kRedoSkip of the items dealt so far have found a
        // pixel above threshold, mark this one without running it: where
        // most items hold such a pixel, the first pass would only add to the
        // second
        int* const s_skip = s_redo + 1;
        if (tid == 0) {
            *s_redo = 0;
            int skip = 0;
            if (blockIdx.x >= kRedoWarm) {
                // set by the item that found the share too large
                skip = __hip_atomic_load(A.redo + kRedoSkipping, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (skip) A.redo[kRedoHead + logical] = 1;
            }
            *s_skip = skip;
        }
        __syncthreads();
        // the same value for every wave: the workgroup leaves as a whole
        if (*s_skip) return;
    }
    CInt* blk = (CInt*)(A.ord + (long long)(byi * A.nvbx + bxi) * A.ord_stride);
    CInt* rec = blk + kCountInts;  // record of the block's k-th frame at rec + k * REC

    float acc[kVPW][kVYW][kRowsW];
#pragma unroll
    for (int q = 0; q < kVPW; ++q)
#pragma unroll
        for (int s = 0; s < kVYW; ++s)
#pragma unroll
            for (int r = 0; r < kRowsW; ++r) acc[q][s][r] = 0.f;

    if constexpr (STAGED) {
        // this wave's staging loads: instructions wave, wave + NW, ... of the
        // NI per frame; lane l of instruction s copies the 16 bytes 64 s + l
        // of the window: 16 / CB columns from column k = (64 s + l) 16 / CB
        // of the window (row group k / CW, column k % CW); lanes past the
        // window copy its first chunk into the buffer's slack
        const int nst = (NI - wave + NW - 1) / NW;
        int voff[NSTX];
#pragma unroll
        for (int j = 0; j < NSTX; ++j) {
            const int k = ((wave + NW * j) * kWave + lane) * (16 / CB);
            voff[j] = k < RG * CW ? ((k / CW) * A.Wp + k % CW) * CB : 0;
        }
        // bytes of the item's origin in a padded frame (a split item's
        // window starts at its row half)
        const int toff = (((Y0 >> 2) + (SPLIT ? 4 * h : 0)) * A.Wp + X0) * CB;
        const int fbytes = (int)(A.fstride * CB / 4);   // < 2^31 on this path
        // frame k of the block into its ring buffer (past the last frame: a
        // repeat of it, never read); the frame's address and float32 window
        // offset from k's record (16-bit copies sit at the same addresses
        // with half the offsets)
        auto stage = [&](int k, int lo, int hi, int woff) __attribute__((always_inline)) {
            const float* fr = reinterpret_cast<const float*>(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
            stage_window<NW, NSTX>(fr, fbytes, voff, nst, (HALF ? woff >> 1 : woff) + toff,
                                   lds + (k % NBUF) * BUFF, wave);
        };
        // the first NBUF - 1 frames (PAIR: the first two)
        constexpr int NPRO = PAIR ? 2 : NBUF - 1;
#pragma unroll
        for (int k = 0; k < NPRO; ++k) {
            const int lo = rec[k * REC], hi = rec[k * REC + 1], woff = rec[k * REC + 2];
            stage(k, lo, hi, woff);
        }
        // this wave's loads of frame 0 (PAIR: of frames 0 and 1) have landed
        if constexpr (PAIR)
            wait_loads<0>();
        else if (nst == NSTX)
            wait_loads<NSTX * (NBUF - 2)>();
        else
            wait_loads<(NSTX - 1) * (NBUF - 2)>();
        barrier_no_fence();
        // records of the next frame to load (rs) and of the frame being added
        // (rc), read one frame ahead (scalar loads, first used after the
        // frame's LDS reads); the block's list has copies of its last record
        // past its end
        CInt* rs = rec + NPRO * REC;
        CInt* rc = rec;
        int slo = rs[0], shi = rs[1], swoff = rs[2];
        // (PAIR: the record of the second frame an even frame stages)
        int s1lo = PAIR ? rs[REC] : 0, s1hi = PAIR ? rs[REC + 1] : 0, s1woff = PAIR ? rs[REC + 2] : 0;
        int cgg = rc[3];
        float csc = HALF ? __int_as_float(rc[kRecScale]) : 1.f;
        int ccol[kVPW];
#pragma unroll
        for (int q = 0; q < kVPW; ++q) ccol[q] = rc[kRecCol + kVPW * xg + q];
        int k = 0;
        auto frame = [&](auto cc) __attribute__((always_inline)) {
            constexpr int C = decltype(cc)::value;
            // frame k + NBUF - 1 into the buffer frame k - 1 used (PAIR:
            // each even frame stages frames k + 2 and k + 3 into the buffers
            // of frames k - 2 and k - 1, which every wave finished before
            // the barrier that ended frame k - 1)
            if constexpr (PAIR) {
                if ((k & 1) == 0) {
                    stage(k + 2, slo, shi, swoff);
                    stage(k + 3, s1lo, s1hi, s1woff);
                }
            } else {
                stage(k + NBUF - 1, slo, shi, swoff);
            }
            if (busy) {
                const T* base = reinterpret_cast<const T*>(lds + (k % NBUF) * BUFF) + (SPLIT ? 0 : 4 * h * CW) + lane;
                if constexpr (item_waves_per_eu(SH, DETECT, DEFER) == 4)
                    add_frame1<C, CW>(base, ccol, cgg & 0xFFFF, cgg >> 16, csc, acc);
                else
                    add_frame<C, CW>(base, ccol, cgg & 0xFFFF, cgg >> 16, csc, acc);
            }
            // next records, loaded after the frame's LDS reads have been
            // used (scalar loads share their wait counter with LDS reads and
            // return out of order: issued earlier, they would turn the
            // partial waits on LDS reads into full ones)
            __builtin_amdgcn_sched_barrier(0);
            rc += REC;
            const int ngg = rc[3];
            const float nsc = HALF ? __int_as_float(rc[kRecScale]) : 1.f;
            int ncol[kVPW];
#pragma unroll
            for (int q = 0; q < kVPW; ++q) ncol[q] = rc[kRecCol + kVPW * xg + q];
            if constexpr (PAIR) {
                if (k & 1) {
                    // records of the two frames the next frame stages; this
                    // wave's loads of frames k + 1 and k + 2 have landed, and
                    // after the barrier everyone's have
                    rs += 2 * REC;
                    const int nlo = rs[0], nhi = rs[1], nwoff = rs[2];
                    const int n1lo = rs[REC], n1hi = rs[REC + 1], n1woff = rs[REC + 2];
                    wait_loads<0>();
                    barrier_no_fence();
                    slo = nlo;
                    shi = nhi;
                    swoff = nwoff;
                    s1lo = n1lo;
                    s1hi = n1hi;
                    s1woff = n1woff;
                }
            } else {
                rs += REC;
                const int nlo = rs[0], nhi = rs[1], nwoff = rs[2];
                // this wave's loads of frame k + 1 have landed; after the
                // barrier, everyone's have
                if (nst == NSTX)
                    wait_loads<NSTX * (NBUF - 2)>();
                else
                    wait_loads<(NSTX - 1) * (NBUF - 2)>();
                barrier_no_fence();
                slo = nlo;
                shi = nhi;
                swoff = nwoff;
            }
            cgg = ngg;
            csc = nsc;
#pragma unroll
            for (int q = 0; q < kVPW; ++q) ccol[q] = ncol[q];
            ++k;
        };
        // one loop per read pattern, in the order the host sorted the frames
        auto loop = [&](auto cc) __attribute__((always_inline)) {
            constexpr int C = decltype(cc)::value;
            const int cnt = blk[C];
#pragma unroll 1
            for (int t = 0; t < cnt; ++t) frame(cc);
        };
        for_cases(loop, std::make_integer_sequence<int, kNCase>{});
        // the repeats issued past the last frame land before LDS is reused
        wait_loads<0>();
        barrier_no_fence();
    } else {
        // Direct path for velocity blocks whose shift spread does not fit the
        // staged window: every sample is read from the padded copy through L2,
        // frames in the block's order.
        typedef const __attribute__((address_space(1))) float GFloat;
        GFloat* pad = (GFloat*)A.pad;
        if (busy) {
            for (int k = 0; k < A.n; ++k) {
                const int i = rec[k * REC + 4];
                const int* rx = A.DX + (long long)i * A.ldx + aw;
                const int* ry = A.DY + (long long)i * A.ldy + b0;
                GFloat* fr = pad + (long long)i * A.fstride;
#pragma unroll
                for (int s = 0; s < kVYW; ++s) {
                    const int yb = Y0 + h * kRowsW + ry[s] + A.padT;
#pragma unroll
                    for (int q = 0; q < kVPW; ++q) {
                        const int xc = X0 + lane + rx[q] + A.padL;
#pragma unroll
                        for (int r = 0; r < kRowsW; ++r) acc[q][s][r] += fr[pad_at(yb + r, xc, A.Wp)];
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
    }

    const int x = X0 + lane;
    const bool xin = x >= 0 && x < A.w;

    // Coverage tables for the epilogue, once per workgroup: the y intervals of
    // the pair's two velocity rows over the tile's rows, the variance prefix
    // (when it fits) and each lane's x intervals.  (sIY and sRS have one row
    // before tile row 0 of the first velocity row, so that a column starting
    // at tile row -1 has a valid base.)
    using L = Lds<SH, NBUF>;
    float* const colarea = lds;
    float* const xch = lds + L::colf;
    int* const sIYa = reinterpret_cast<int*>(xch + L::xch);
    float* const sRSa = reinterpret_cast<float*>(sIYa + L::iy);
    float* const sRM = sRSa + L::rs;
    float* const sCB = sRM + L::rm;
    double* const sP = reinterpret_cast<double*>(sCB + L::cb);
    int* const sIY = sIYa + 2;
    float* const sRS = sRSa + 1;
    const bool need_c = DETECT || A.mean || A.cov != nullptr;
    int xlo[kVPW], xhi[kVPW];
#pragma unroll
    for (int q = 0; q < kVPW; ++q) {
        xlo[q] = A.n;
        xhi[q] = -1;
        if (need_c && xin && aw + q < A.nvx) load_iv(A.IX, (long long)(aw + q) * A.w + x, xlo[q], xhi[q]);
    }
    if (need_c) {
        for (int e = tid; e < kVYW * kRows; e += NW * kWave) {
            const int bb = b0 + e / kRows, y = Y0 + e % kRows;
            int lo = A.n, hi = -1;
            if (bb < A.nvy && y >= 0 && y < A.h) load_iv(A.IY, (long long)bb * A.h + y, lo, hi);
            sIY[2 * e] = lo;
            sIY[2 * e + 1] = hi;
        }
    }
    const bool p_lds = DETECT && A.n + 1 <= kPLds;
    if (DETECT) {
        if (p_lds)
            for (int e = tid; e <= A.n; e += NW * kWave) sP[e] = A.P[e];
        // per (velocity row, tile row): 1/sqrt(V) over the row's y interval
        for (int e = tid; e < kVYW * kRows; e += NW * kWave) {
            const int bb = b0 + e / kRows, y = Y0 + e % kRows;
            int lo = A.n, hi = -1;
            if (bb < A.nvy && y >= 0 && y < A.h) load_iv(A.IY, (long long)bb * A.h + y, lo, hi);
            float rs = 0.f;
            if (hi >= lo) {
                const double V = A.P[hi + 1] - A.P[lo];
                rs = V > 0.0 ? rsqrtf((float)V) : 0.f;
            }
            sRS[e] = rs;
            sRM[e] = (hi - lo + 1 >= A.cmin && hi >= lo) ? rs : __builtin_nanf("");
            // 16-bit samples: the backgrounds of the row's frames, subtracted
            // from sums whose x samples all lie inside
            if constexpr (HALF) sCB[e] = hi >= lo ? (float)(A.Pb[hi + 1] - A.Pb[lo]) : 0.f;
        }
    }
    // publish the row next to the other half: row kRowsW - 1 of the upper
    // half, row 0 of the lower one (after the background of the 16-bit
    // search, which needs the tables, is subtracted)
    auto publish = [&]() __attribute__((always_inline)) {
        float* xo = xch + wave * (kVPW * kVYW * kWave);
#pragma unroll
        for (int q = 0; q < kVPW; ++q)
#pragma unroll
            for (int s = 0; s < kVYW; ++s) xo[(q * kVYW + s) * kWave + lane] = h ? acc[q][s][0] : acc[q][s][kRowsW - 1];
    };
    if constexpr (DETECT && !HALF && !SPLIT) publish();
    if (need_c) __syncthreads();
    // 16-bit samples: S' = sum of scale * sample - the covering frames'
    // means, their sum from the prefix of the means (the S/N evaluation of
    // a single pixel does the same); for a lane whose x samples all lie
    // inside, the covering frames are the row's, whose sum is tabulated
    auto bg_row = [&](int q, int e) __attribute__((always_inline)) -> float {
        if (xlo[q] == 0 && xhi[q] == A.n - 1) return sCB[e];
        int lo, hi;
        const int cv = coverage(xlo[q], xhi[q], sIY[2 * e], sIY[2 * e + 1], lo, hi);
        return cv > 0 ? (float)(A.Pb[hi + 1] - A.Pb[lo]) : 0.f;
    };
    if constexpr (HALF && !SPLIT) {
        float* xo = xch + wave * (kVPW * kVYW * kWave);
#pragma unroll
        for (int q = 0; q < kVPW; ++q)
#pragma unroll
            for (int s = 0; s < kVYW; ++s) {
                const int r = h ? 0 : kRowsW - 1;
                xo[(q * kVYW + s) * kWave + lane] = acc[q][s][r] - bg_row(q, s * kRows + h * kRowsW + r);
            }
        __syncthreads();
    }

    if constexpr (!DETECT) {
        // plain stack: SUM or MEAN, optional coverage
        auto value = [&](int q, int s, int r, int& c) __attribute__((always_inline)) -> float {
            float v = acc[q][s][r];
            c = 0;
            if (need_c) {
                int lo, hi;
                const int tr = h * kRowsW + r;
                c = max(0, coverage(xlo[q], xhi[q], sIY[2 * (s * kRows + tr)], sIY[2 * (s * kRows + tr) + 1], lo, hi));
            }
            if (A.mean) v = c > 0 ? v / (float)c : 0.f;
            return v;
        };
        // A tile inside the frame's columns (row length a multiple of four,
        // outputs 16-byte aligned) writes each velocity's 16 x 64 block of
        // the wave through the wave's LDS column area, so that a lane stores
        // four adjacent columns of one row with one 16-byte store: four times
        // fewer store instructions, which keeps the stores from holding the
        // workgroup long after its frame loop.  Streaming stores: the stacks
        // are not read again by this kernel, the staged frames are.
        const bool wide = X0 + kTileW <= A.w && (A.w & 3) == 0 && ((uintptr_t)A.out & 15) == 0 &&
                          ((uintptr_t)A.cov & 15) == 0;
        if (wide) {
            float* tb = colarea + wave * (kColRows * kWave);
            const int rr = lane >> 4, cc = (lane & 15) * 4;
            if (!need_c) {
                // SUM without coverage (its own loop: no per-element
                // coverage code to schedule around)
#pragma unroll
                for (int q = 0; q < kVPW; ++q) {
#pragma unroll
                    for (int s = 0; s < kVYW; ++s) {
                        const int a = aw + q, bb = b0 + s;
                        if (a < A.nvx && bb < A.nvy) {
                            const long long base = ((long long)bb * A.nvx + a) * A.h;
#pragma unroll
                            for (int r = 0; r < kRowsW; ++r) tb[r * kWave + lane] = acc[q][s][r];
#pragma unroll
                            for (int j = 0; j < kRowsW / 4; ++j) {
                                const int y = Y0 + h * kRowsW + 4 * j + rr;
                                const f4 v = *reinterpret_cast<const f4*>(tb + (4 * j + rr) * kWave + cc);
                                if (y < A.h)
                                    __builtin_nontemporal_store(
                                        v, reinterpret_cast<f4*>(A.out + (base + y) * A.w + X0 + cc));
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                return;
            }
#pragma unroll
            for (int q = 0; q < kVPW; ++q) {
#pragma unroll
                for (int s = 0; s < kVYW; ++s) {
                    const int a = aw + q, bb = b0 + s;
                    if (a < A.nvx && bb < A.nvy) {
                        const long long base = ((long long)bb * A.nvx + a) * A.h;
#pragma unroll
                        for (int r = 0; r < kRowsW; ++r) {
                            int c;
                            tb[r * kWave + lane] = value(q, s, r, c);
                        }
#pragma unroll
                        for (int j = 0; j < kRowsW / 4; ++j) {
                            const int y = Y0 + h * kRowsW + 4 * j + rr;
                            const f4 v = *reinterpret_cast<const f4*>(tb + (4 * j + rr) * kWave + cc);
                            if (y < A.h)
                                __builtin_nontemporal_store(v, reinterpret_cast<f4*>(A.out + (base + y) * A.w + X0 + cc));
                        }
                        if (A.cov) {
#pragma unroll
                            for (int r = 0; r < kRowsW; ++r) {
                                int c;
                                (void)value(q, s, r, c);
                                tb[r * kWave + lane] = __int_as_float(c);
                            }
#pragma unroll
                            for (int j = 0; j < kRowsW / 4; ++j) {
                                const int y = Y0 + h * kRowsW + 4 * j + rr;
                                const i4 c = *reinterpret_cast<const i4*>(tb + (4 * j + rr) * kWave + cc);
                                if (y < A.h)
                                    __builtin_nontemporal_store(
                                        c, reinterpret_cast<i4*>(A.cov + (base + y) * A.w + X0 + cc));
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            return;
        }
        if (!xin) return;
#pragma unroll
        for (int q = 0; q < kVPW; ++q) {
#pragma unroll
            for (int s = 0; s < kVYW; ++s) {
                const int a = aw + q, bb = b0 + s;
                if (a < A.nvx && bb < A.nvy) {
                    const long long kk = (long long)bb * A.nvx + a;
#pragma unroll
                    for (int r = 0; r < kRowsW; ++r) {
                        const int y = Y0 + h * kRowsW + r;
                        if (y < A.h) {
                            int c;
                            const float v = value(q, s, r, c);
                            const long long o = (kk * A.h + y) * A.w + x;
                            __builtin_nontemporal_store(v, A.out + o);
                            if (A.cov) __builtin_nontemporal_store(c, A.cov + o);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        return;
    } else {
        // written out per velocity (not a loop) so that acc stays in
        // registers: the epilogue is too large for the unroller to replicate
        float* col = colarea + wave * (kColRows * kWave);
        const float* xin_rows = SPLIT ? nullptr : xch + (wave ^ 1) * (kVPW * kVYW * kWave);
        const int R0 = kRowsW * h - 1;
        auto one = [&](auto qc, auto sc, const double* P) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value, s = decltype(sc)::value;
            const int bb = b0 + s;
            if (aw + q < A.nvx && bb < A.nvy) {
                if constexpr (HALF) {
                    const int e0 = s * kRows + h * kRowsW;
                    if (__ballot(!(xlo[q] == 0 && xhi[q] == A.n - 1)) == 0) {
                        const f4* cb = reinterpret_cast<const f4*>(sCB + e0);
#pragma unroll
                        for (int k = 0; k < kRowsW / 4; ++k) {
                            const f4 t = cb[k];
                            acc[q][s][4 * k] -= t.x;
                            acc[q][s][4 * k + 1] -= t.y;
                            acc[q][s][4 * k + 2] -= t.z;
                            acc[q][s][4 * k + 3] -= t.w;
                        }
                    } else {
                        // (a runtime loop through the wave's column area keeps
                        // the registers few)
#pragma unroll 1
                        for (int r = 0; r < kRowsW; ++r) col[r * kWave + lane] = bg_row(q, e0 + r);
#pragma unroll
                        for (int r = 0; r < kRowsW; ++r) acc[q][s][r] -= col[r * kWave + lane];
                    }
                }
                float rsm[kRowsW];  // this row half's multipliers (uniform)
                const f4* src = reinterpret_cast<const f4*>(sRM + s * kRows + h * kRowsW);
#pragma unroll
                for (int k = 0; k < kRowsW / 4; ++k) {
                    const f4 t = src[k];
                    rsm[4 * k] = t.x;
                    rsm[4 * k + 1] = t.y;
                    rsm[4 * k + 2] = t.z;
                    rsm[4 * k + 3] = t.w;
                }
                detect_epilogue<SPLIT, DEFER>(A, Ap, acc[q][s], rsm, aw + q, bb, x, xin, lane, h, Y0, tile, col,
                                SPLIT ? nullptr : xin_rows + (q * kVYW + s) * kWave, sIY + (s * kRows + R0) * 2,
                                sRS + s * kRows + R0,
                                P, xlo[q], xhi[q], VBX, REC, s_redo);
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        auto epi = [&](const double* P) __attribute__((always_inline)) {
            one(ic<0>{}, ic<0>{}, P);
            one(ic<0>{}, ic<1>{}, P);
            one(ic<1>{}, ic<0>{}, P);
            one(ic<1>{}, ic<1>{}, P);
            one(ic<2>{}, ic<0>{}, P);
            one(ic<2>{}, ic<1>{}, P);
        };
        static_assert(kVPW == 3 && kVYW == 2, "one call per velocity of the wave");
        // two instantiations so that the common one reads the prefix from LDS
        if (p_lds)
            epi(sP);
        else
            epi(A.P);
        if constexpr (DEFER) {
            // mark the item for the second pass if a wave found a pixel above
            // threshold (0 otherwise: every item of the grid is written);
            // the count covers the items this pass ran
            __syncthreads();
            if (tid == 0) {
                const int found = *s_redo;
                A.redo[kRedoHead + logical] = found;
                if (found) {
                    const int seen = atomicAdd(A.redo + kRedoFound, 1) + 1;
                    if ((int)blockIdx.x >= kRedoWarm && seen * kRedoSkip > (int)blockIdx.x)
                        __hip_atomic_store(A.redo + kRedoSkipping, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

// (the plain stack of shape 2 and the first pass of its two-pass search fit
// the registers of four waves per SIMD, which lets four workgroups share a CU)
template <bool DETECT, bool STAGED, int SH, bool HALF, bool DEFER = false>
__global__ __launch_bounds__(shape_waves(SH) * kWave)
__attribute__((amdgpu_waves_per_eu(item_waves_per_eu(SH, DETECT, DEFER))))
void k_stack(const StackArgs A) {
    __shared__ __attribute__((aligned(16))) float lds[Lds<SH, item_nbuf(SH, DETECT, DEFER)>::total];
    stack_item<DETECT, STAGED, SH, HALF, DEFER>(A, (KArgs)__builtin_amdgcn_kernarg_segment_ptr(),
                                                xcd_remap(blockIdx.x, gridDim.x), lds);
}

// Between the passes of a two-pass search: the G work items the first pass
// marked, listed in increasing order. Workgroup c handles the kCompactChunk
// marks from c kCompactChunk, four consecutive ones per thread: the first
// kernel counts each chunk's marks, the second adds up the counts of the
// chunks before its own and lists its items from there.
__device__ __forceinline__ int compact_marks(const int* __restrict__ redo, int G, int i0, int m[4]) {
    const int* mark = redo + kRedoHead;
    if (i0 + 3 < G) {
        // kRedoHead and i0 are multiples of four: an aligned 16-byte load
        const int4 v = *reinterpret_cast<const int4*>(mark + i0);
        m[0] = v.x;
        m[1] = v.y;
        m[2] = v.z;
        m[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] = i0 + k < G ? mark[i0 + k] : 0;
    }
    return (m[0] != 0) + (m[1] != 0) + (m[2] != 0) + (m[3] != 0);
}

// inclusive sum over the workgroup's threads up to this one; *all: the sum
// over all of them
__device__ __forceinline__ int compact_scan(int c, int* wsum, int* all) {
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
    int x = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wv] = x;
    __syncthreads();
    int before = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kCompactThreads / kWave; ++k) {
        before += k < wv ? wsum[k] : 0;
        sum += wsum[k];
    }
    __syncthreads();
    *all = sum;
    return before + x;
}

__global__ __launch_bounds__(kCompactThreads) void k_redo_count(int* __restrict__ redo, int G) {
    __shared__ int wsum[kCompactThreads / kWave];
    int m[4], all;
    const int c = compact_marks(redo, G, blockIdx.x * kCompactChunk + 4 * threadIdx.x, m);
    compact_scan(c, wsum, &all);
    if (threadIdx.x == 0) redo[kRedoHead + 2 * G + blockIdx.x] = all;
}

__global__ __launch_bounds__(kCompactThreads) void k_redo_list(int* __restrict__ redo, int G) {
    __shared__ int wsum[kCompactThreads / kWave];
    const int* counts = redo + kRedoHead + 2 * G;
    int base = 0, all;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kCompactThreads) base += counts[k];
    compact_scan(base, wsum, &all);
    base = all;
    int m[4];
    const int i0 = blockIdx.x * kCompactChunk + 4 * threadIdx.x;
    const int c = compact_marks(redo, G, i0, m);
    int off = base + compact_scan(c, wsum, &all) - c;
    int* list = redo + kRedoHead + G;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (m[k]) list[off++] = i0 + k;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) redo[kRedoTotal] = base + all;
}

// Second pass of a two-pass search: the listed items, run in full
// (candidates included). The list is cut into kRedoRuns equal runs, and the
// workgroups dealt to XCD x (blockIdx.x % kRedoRuns) take run x in order, so
// that items that lie close together run on one XCD, as in the first pass;
// the grid is the first pass's rounded up to a multiple of kRedoRuns (every
// run's workgroups exist), and workgroups past the runs exit at once.
template <int SH>
__global__ __launch_bounds__(shape_waves(SH) * kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_stack_redo(const StackArgs A, int G) {
    __shared__ __attribute__((aligned(16))) float lds[Lds<SH, item_nbuf(SH, true, false)>::total];
    const int total = A.redo[kRedoTotal];
    const int per = (total + kRedoRuns - 1) / kRedoRuns;
    const int r = blockIdx.x / kRedoRuns;
    const int j = (blockIdx.x % kRedoRuns) * per + r;
    if (r >= per || j >= total) return;
    const int logical = A.redo[kRedoHead + G + j];
    stack_item<true, true, SH>(A, (KArgs)__builtin_amdgcn_kernarg_segment_ptr(), logical, lds);
}

// Persistent form for a batch of detect problems (all staged): each
// workgroup takes work items from its queue until the queue is empty, then
// helps the other queues; an item is a (tile, velocity block) of one
// problem, found by binary search of the problems' first items.
template <int SH>
__global__ __launch_bounds__(shape_waves(SH) * kWave) __attribute__((amdgpu_waves_per_eu(3)))
void k_stack_batch(const BatchArgs B) {
    // the table is read-only during the launch: read it through the constant
    // address space, so that the (uniform) loads are scalar
    typedef const __attribute__((address_space(4))) StackArgs CArgs;
    __shared__ __attribute__((aligned(16))) float lds[Lds<SH, item_nbuf(SH, true, false)>::total];
    int* const s_item = reinterpret_cast<int*>(lds + Lds<SH, item_nbuf(SH, true, false)>::total - 4);
    const int q0 = blockIdx.x % kBatchQueues;
    // the workgroup's own queue first, then (for the tail of the launch)
    // the other queues in turn; every queue ends, so every workgroup exits
    for (int k = 0; k < kBatchQueues; ++k) {
        const int q = (q0 + k) % kBatchQueues;
        const int begin = B.qbegin[q], end = B.qbegin[q + 1];
        for (;;) {
            if (threadIdx.x == 0) *s_item = begin + atomicAdd(B.counter + q, 1);
            __syncthreads();
            const int g = __builtin_amdgcn_readfirstlane(*s_item);
            __syncthreads();
            if (g >= end) break;
            int lo = 0, hi = B.nprob - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (B.start[mid] <= g)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const StackArgs* Ap = (const StackArgs*)((CArgs*)B.tab + lo);
            stack_item<true, true, SH>(*Ap, Ap, g - B.start[lo], lds);
            // every wave has finished the item before the next one reuses LDS
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kAux) void k_zero_i32(int* __restrict__ p, int count) {
    const int i = blockIdx.x * kAux + threadIdx.x;
    if (i < count) p[i] = 0;
}

// ------------------------------------------------------------------ merge
// One workgroup per velocity: gather the entries kept by every tile, rank
// them by key and write the first k_max in order; count = all candidates.
__device__ __forceinline__ void merge(const int32_t* __restrict__ tcount, const Entry* __restrict__ ent, int nslot,
                                      int kt, int k_max, int nvx, int w, int k_first, sst_candidate* __restrict__ cand,
                                      int32_t* __restrict__ count, int* __restrict__ flag, int kc) {
    const int k = k_first + kc;
    __shared__ unsigned long long keys[kMergeLds];
    __shared__ int idx[kMergeLds];
    __shared__ int nst;
    __shared__ unsigned long long last;  // key of the list's k_max-th entry (0: fewer than k_max)
    __shared__ int inexact;
    __shared__ long long shl[4];
    __shared__ unsigned long long bk[4];
    __shared__ long long bi[4];
    if (threadIdx.x == 0) {
        nst = 0;
        last = 0;
        inexact = 0;
    }
    __syncthreads();
    const int32_t* tc = tcount + (long long)kc * nslot;
    const Entry* E = ent + (long long)kc * nslot * kt;
    long long tot = 0;
    for (int t = threadIdx.x; t < nslot; t += kAux) {
        const int c = tc[t];
        tot += c;
        const int s = min(c, kt);
        for (int e = 0; e < s; ++e) {
            const int slot = atomicAdd(&nst, 1);
            if (slot < kMergeLds) {
                const Entry en = E[(long long)t * kt + e];
                keys[slot] = cand_key(en.sn, en.raster);
                idx[slot] = t * kt + e;
            }
        }
    }
    tot = block_sum_i64(tot, shl);  // contains barriers: LDS gathers are complete
    const int m = nst;
    const int nout = min(k_max, m);
    sst_candidate* out = cand + (long long)k * k_max;
    const int ivx = k % nvx, ivy = k / nvx;
    auto emit = [&](const Entry& en, int r) {
        sst_candidate o;
        o.ivx = ivx;
        o.ivy = ivy;
        o.x = en.raster % w;
        o.y = en.raster / w;
        o.snr = en.sn;
        o.flux = en.flux;
        o.coverage = en.cov;
        o.rank = r;
        out[r] = o;
    };
    if (m <= kMergeLds) {
        for (int e = threadIdx.x; e < m; e += kAux) {
            const unsigned long long ke = keys[e];
            int r = 0;
            for (int f = 0; f < m; ++f) r += keys[f] > ke ? 1 : 0;
            if (r < k_max) emit(E[idx[e]], r);
            if (r == k_max - 1) last = ke;
        }
    } else {
        unsigned long long prev = ~0ull;
        for (int r = 0; r < nout; ++r) {
            unsigned long long best = 0;
            long long bidx = -1;
            for (int t = threadIdx.x; t < nslot; t += kAux) {
                const int s = min(tc[t], kt);
                for (int e = 0; e < s; ++e) {
                    const Entry en = E[(long long)t * kt + e];
                    const unsigned long long key = cand_key(en.sn, en.raster);
                    if (key < prev && key > best) {
                        best = key;
                        bidx = (long long)t * kt + e;
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long tk = __shfl_xor(best, o);
                const long long ti = __shfl_xor(bidx, o);
                if (tk > best) {
                    best = tk;
                    bidx = ti;
                }
            }
            if ((threadIdx.x & 63) == 0) {
                bk[threadIdx.x >> 6] = best;
                bi[threadIdx.x >> 6] = bidx;
            }
            __syncthreads();
            unsigned long long gb = bk[0];
            long long gi = bi[0];
            for (int wv = 1; wv < 4; ++wv)
                if (bk[wv] > gb) {
                    gb = bk[wv];
                    gi = bi[wv];
                }
            if (threadIdx.x == 0) emit(E[gi], r);
            prev = gb;
            __syncthreads();
        }
        if (threadIdx.x == 0 && nout == k_max) last = prev;
    }
    // A slot that found more candidates than it kept dropped only keys below
    // its last kept one; the list is exact unless such a key could rank
    // among the first k_max.  Otherwise the velocity is listed for an exact
    // recomputation.
    __syncthreads();
    for (int t = threadIdx.x; t < nslot; t += kAux)
        if (tc[t] > kt) {
            const Entry en = E[(long long)t * kt + kt - 1];
            if (cand_key(en.sn, en.raster) > last) inexact = 1;
        }
    __syncthreads();
    if (threadIdx.x == 0 && inexact) flag[kFlagHead + atomicAdd(flag, 1)] = kc;
    for (int r = nout + threadIdx.x; r < k_max; r += kAux) {
        sst_candidate o;
        o.ivx = ivx;
        o.ivy = ivy;
        o.x = -1;
        o.y = -1;
        o.snr = -INFINITY;
        o.flux = 0.f;
        o.coverage = 0;
        o.rank = -1;
        out[r] = o;
    }
    if (threadIdx.x == 0) count[k] = (int32_t)min(tot, (long long)INT_MAX);
}

__global__ __launch_bounds__(kAux) void k_merge(const int32_t* __restrict__ tcount, const Entry* __restrict__ ent,
                                                   int nslot, int kt, int k_max, int nvx, int w, int k_first,
                                                   sst_candidate* __restrict__ cand, int32_t* __restrict__ count,
                                                   int* __restrict__ flag) {
    merge(tcount, ent, nslot, kt, k_max, nvx, w, k_first, cand, count, flag, blockIdx.x);
}

// ------------------------------------------------- batched preparation
// The same kernels for every plan of a batch in one launch each: workgroup
// t belongs to the job j with off[j] <= t < off[j + 1] and runs that job's
// workgroup t - off[j] (in the order of the single-plan grid, x fastest).
__device__ __forceinline__ int job_of(const int* __restrict__ off, int np, int t) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kAux) void k_stats_partial_batch(const PrepBatch B) {
    const int t = blockIdx.x;
    const int j = job_of(B.off, B.np, t);
    const PrepJob& J = B.jobs[j];
    const int l = t - B.off[j];
    const int i = l / J.nchunk, c = l - i * J.nchunk;
    if (B.dtype[j] == SST_BF16)
        stats_partial<SST_BF16>(B.frames[j], B.scale[j], J.npx, J.nchunk, J.part, i, c);
    else if (B.dtype[j] == SST_F16)
        stats_partial<SST_F16>(B.frames[j], B.scale[j], J.npx, J.nchunk, J.part, i, c);
    else
        stats_partial<SST_F32>(B.frames[j], B.scale[j], J.npx, J.nchunk, J.part, i, c);
}

__global__ __launch_bounds__(kAux) void k_stats_final_batch(const PrepBatch B) {
    const PrepJob& J = B.jobs[blockIdx.x];
    stats_final(J.part, J.nchunk, J.pa.n, J.npx, J.b, J.s2, J.b32, J.P, J.Pb, nullptr);
}

__global__ __launch_bounds__(kAux) void k_prep_batch(const PrepBatch B) {
    const int t = blockIdx.x;
    const int j = job_of(B.off + (B.np + 1), B.np, t);
    const PrepJob& J = B.jobs[j];
    const int l = t - B.off[(B.np + 1) + j];
    const int i = l / J.prep_bx, bx = l - i * J.prep_bx;
    PrepArgs a = J.pa;
    a.frames = B.frames[j];
    a.dtype = B.dtype[j];
    a.scale = B.scale[j];
    if (a.dtype == SST_BF16)
        prep<SST_BF16>(a, i, bx);
    else if (a.dtype == SST_F16)
        prep<SST_F16>(a, i, bx);
    else
        prep<SST_F32>(a, i, bx);
}

// both coverage tables of every job: x (nvx rows of w) then y (nvy rows of h)
__global__ __launch_bounds__(kAux) void k_cov_batch(const PrepBatch B) {
    const int t = blockIdx.x;
    const int j = job_of(B.off + 2 * (B.np + 1), B.np, t);
    const PrepJob& J = B.jobs[j];
    int l = t - B.off[2 * (B.np + 1) + j];
    const int bxx = (J.w + kAux - 1) / kAux, bxy = (J.h + kAux - 1) / kAux;
    if (l < bxx * J.nvx) {
        const int a = l / bxx;
        cov(J.DX, J.ldx, J.pa.n, J.w, J.IX, a, l - a * bxx);
    } else {
        l -= bxx * J.nvx;
        const int b = l / bxy;
        cov(J.DY, J.ldy, J.pa.n, J.h, J.IY, b, l - b * bxy);
    }
}

__global__ __launch_bounds__(kAux) void k_merge_batch(const MergeBatch B) {
    const int t = blockIdx.x;
    const int j = job_of(B.off, B.np, t);
    const MergeJob& J = B.jobs[j];
    merge(J.tcount, J.ent, J.nslot, J.kt, J.k_max, J.nvx, J.w, J.k_first, B.cand[j], B.count[j], J.flag,
          t - B.off[j]);
}

hipError_t launch_prep_batch(const PrepBatch& b, const int* blocks, hipStream_t s) {
    if (b.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats_partial_batch, dim3((unsigned)blocks[0]), dim3(kAux), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final_batch, dim3((unsigned)b.np), dim3(kAux), 0, s, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_prep_batch, dim3((unsigned)blocks[1]), dim3(kAux), 0, s, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cov_batch, dim3((unsigned)blocks[2]), dim3(kAux), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_merge_batch(const MergeBatch& b, int blocks, hipStream_t s) {
    if (b.np <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_batch, dim3((unsigned)blocks), dim3(kAux), 0, s, b);
    return hipGetLastError();
}

// ------------------------------------------------ exact recomputation
// For a listed velocity (its slots kept fewer entries than the k_max best
// may need): a list of the best keys so far in LDS, fed with the kept
// entries of every slot that kept all its candidates and with the
// candidates of every other slot recomputed from the padded copy (the
// stacking loop's float32 sums in the block's frame order, then the same
// S/N, threshold, coverage and 8-neighbour rules on the slot's 16 x 64
// pixels with a border of one), then written over the velocity's list.
constexpr int kFixCap = 2048;         // list entries in LDS
constexpr int kFixRows = kRowsW + 2;  // slot rows with their border
constexpr int kFixCols = kTileW + 2;
constexpr int kFixPix = kFixRows * kFixCols;
constexpr int kFixPer = (kFixPix + kAux - 1) / kAux;  // pixels per thread
constexpr int kSlotMax = (kRowsW / 2) * (kTileW / 2);  // candidates a slot can hold (no two adjacent)

struct FixLds {
    unsigned long long key[kFixCap];
    float flux[kFixCap];
    int cov[kFixCap];
    float sn[kFixPix];
    float acc[kFixPix];
    int c[kFixPix];
    int m;
    int item;
};

// Sort the list descending by key and keep its first `keep` entries.
__device__ void fix_compact(FixLds& L, int keep) {
    __syncthreads();
    const int m = L.m;
    int N = 1;
    while (N < m) N <<= 1;
    for (int i = m + threadIdx.x; i < N; i += kAux) L.key[i] = 0;
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N; i += kAux) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = L.key[i], b = L.key[l];
                    if ((i & k) == 0 ? a < b : a > b) {
                        L.key[i] = b;
                        L.key[l] = a;
                        const float f = L.flux[i];
                        L.flux[i] = L.flux[l];
                        L.flux[l] = f;
                        const int c = L.cov[i];
                        L.cov[i] = L.cov[l];
                        L.cov[l] = c;
                    }
                }
            }
            __syncthreads();
        }
    if (threadIdx.x == 0) L.m = min(m, keep);
    __syncthreads();
}

__device__ __forceinline__ void fix_append(FixLds& L, unsigned long long key, float flux, int cov) {
    const int p = atomicAdd(&L.m, 1);
    L.key[p] = key;
    L.flux[p] = flux;
    L.cov[p] = cov;
}

// The candidates of slot t of velocity (a, b), appended to the list (which
// has room for kSlotMax more).
__device__ void fix_slot(KArgs A, FixLds& L, int a, int b, int t, int vbx, int rec) {
    const int tile = t >> 1, hh = t & 1;
    const int X0 = (tile % A->tiles_x) * kTileW, Y0 = (tile / A->tiles_x) * kRows;
    const int xr = X0 - 1, yr = Y0 + kRowsW * hh - 1;  // pixel of border entry (0, 0)
    const int n = A->n, w = A->w, h = A->h;
    typedef const __attribute__((address_space(1))) float GFloat;
    typedef const __attribute__((address_space(1))) _Float16 GHalf;
    typedef const __attribute__((address_space(1))) int GInt;
    typedef const __attribute__((address_space(1))) double GDouble;
    GInt* ordr = (GInt*)(A->ord + (long long)((b / kVYW) * A->nvbx + a / vbx) * A->ord_stride + kCountInts);
    GInt* DX = (GInt*)A->DX;
    GInt* DY = (GInt*)A->DY;
    const long long fstride = A->fstride;
    float acc[kFixPer];
    int px[kFixPer], py[kFixPer];
    bool in[kFixPer];
#pragma unroll
    for (int q = 0; q < kFixPer; ++q) {
        const int p = threadIdx.x + q * kAux;
        px[q] = xr + p % kFixCols;
        py[q] = yr + p / kFixCols;
        in[q] = p < kFixPix && px[q] >= 0 && px[q] < w && py[q] >= 0 && py[q] < h;
        acc[q] = 0.f;
    }
    // the sums, frame by frame in the block's order
    for (int k = 0; k < n; ++k) {
        const int i = ordr[(long long)k * rec + 4];
        const int dx = DX[(long long)i * A->ldx + a] + A->padL, dy = DY[(long long)i * A->ldy + b] + A->padT;
        if (A->half) {
            GHalf* pad16 = (GHalf*)A->pad + 2 * (long long)i * fstride;
            const float sc = ((GFloat*)A->scale)[i];
#pragma unroll
            for (int q = 0; q < kFixPer; ++q)
                if (in[q]) acc[q] = __builtin_fmaf((float)pad16[pad_at(py[q] + dy, px[q] + dx, A->Wp)], sc, acc[q]);
        } else {
            GFloat* pad = (GFloat*)A->pad + (long long)i * fstride;
#pragma unroll
            for (int q = 0; q < kFixPer; ++q)
                if (in[q]) acc[q] += pad[pad_at(py[q] + dy, px[q] + dx, A->Wp)];
        }
    }
    // S/N and coverage, as the stacking kernel forms them
    const double* P = A->P;
#pragma unroll
    for (int q = 0; q < kFixPer; ++q) {
        const int p = threadIdx.x + q * kAux;
        if (p >= kFixPix) continue;
        float sn = -INFINITY, v = acc[q];
        int cov = 0;
        if (in[q]) {
            int xlo, xhi, ylo, yhi, lo, hi;
            load_iv(A->IX, (long long)a * w + px[q], xlo, xhi);
            load_iv(A->IY, (long long)b * h + py[q], ylo, yhi);
            cov = coverage(xlo, xhi, ylo, yhi, lo, hi);
            if (cov > 0) {
                if (A->half) v -= (float)(((GDouble*)A->Pb)[hi + 1] - ((GDouble*)A->Pb)[lo]);
                const double V = P[hi + 1] - P[lo];
                if (xlo == 0 && xhi == n - 1) {
                    sn = v * (V > 0.0 ? rsqrtf((float)V) : 0.f);
                } else {
                    sn = V > 0.0 ? v * rsqrtf((float)V) : 0.f;
                }
            }
        }
        L.sn[p] = sn;
        L.acc[p] = v;
        L.c[p] = cov;
    }
    __syncthreads();
    // peaks of the slot's own pixels (border entries 1 .. kFixRows - 2 and
    // 1 .. kFixCols - 2): above threshold with enough coverage, above every
    // earlier neighbour in raster order and not below any later one
    for (int e = threadIdx.x; e < kRowsW * kTileW; e += kAux) {
        const int r = 1 + e / kTileW, cc = 1 + e % kTileW;
        const int p = r * kFixCols + cc;
        const float sv = L.sn[p];
        if (!(L.c[p] >= A->cmin && sv > A->thr)) continue;
        bool ok = true;
        for (int k = 0; k < 9 && ok; ++k) {
            if (k == 4) continue;
            const int dy = k / 3 - 1, dx = k % 3 - 1;
            const float sq = L.sn[p + dy * kFixCols + dx];
            ok = (dy < 0 || (dy == 0 && dx < 0)) ? sv > sq : sv >= sq;
        }
        if (ok) {
            const int x = xr + cc, y = yr + r;
            fix_append(L, cand_key(sv, y * w + x), L.acc[p], L.c[p]);
        }
    }
    __syncthreads();
}

// Exact list of velocity kc of a merge job (A: the launch's arguments).
__device__ void fix_velocity(KArgs A, const MergeJob& J, sst_candidate* cand, FixLds& L, int kc) {
    const int k = J.k_first + kc;
    const int a = k % J.nvx, b = k / J.nvx;
    const int32_t* tc = J.tcount + (long long)kc * J.nslot;
    const Entry* E = J.ent + (long long)kc * J.nslot * J.kt;
    if (threadIdx.x == 0) L.m = 0;
    __syncthreads();
    for (int t = 0; t < J.nslot; ++t) {
        const int c = tc[t];  // (uniform)
        if (c == 0) continue;
        const int add = c <= J.kt ? c : kSlotMax;
        if (L.m + add > kFixCap) fix_compact(L, J.k_max);
        if (c <= J.kt) {
            for (int e = threadIdx.x; e < c; e += kAux) {
                const Entry en = E[(long long)t * J.kt + e];
                fix_append(L, cand_key(en.sn, en.raster), en.flux, en.cov);
            }
            __syncthreads();
        } else {
            fix_slot(A, L, a, b, t, J.vbx, J.rec);
        }
    }
    fix_compact(L, J.k_max);
    sst_candidate* out = cand + (long long)k * J.k_max;
    for (int r = threadIdx.x; r < J.k_max; r += kAux) {
        sst_candidate o;
        o.ivx = a;
        o.ivy = b;
        if (r < L.m) {
            const unsigned long long key = L.key[r];
            unsigned u = (unsigned)(key >> 32);
            u ^= (u & 0x80000000u) ? 0x80000000u : 0xFFFFFFFFu;
            const int raster = (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
            o.x = raster % J.w;
            o.y = raster / J.w;
            o.snr = __uint_as_float(u);
            o.flux = L.flux[r];
            o.coverage = L.cov[r];
            o.rank = r;
        } else {
            o.x = -1;
            o.y = -1;
            o.snr = -INFINITY;
            o.flux = 0.f;
            o.coverage = 0;
            o.rank = -1;
        }
        out[r] = o;
    }
    __syncthreads();
}

// The listed velocities of jobs [0, njobs), taken one at a time; the last
// workgroup to finish clears every job's list.
template <typename GetJob>
__device__ void fix_loop(int njobs, GetJob get) {
    __shared__ FixLds L;
    __shared__ int listed;
    int* head = get(0).flag;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int j = 0; j < njobs; ++j) any |= atomicAdd(get(j).flag, 0);
        listed = any;
    }
    __syncthreads();
    if (listed == 0) return;  // no velocity listed by these merges (the same in every workgroup)
    for (int j = 0; j < njobs; ++j) {
        KArgs A;
        sst_candidate* cand;
        const MergeJob& J = get(j, &A, &cand);
        for (;;) {
            if (threadIdx.x == 0) {
                const int it = atomicAdd(J.flag + 1, 1);
                L.item = it < atomicAdd(J.flag, 0) ? J.flag[kFlagHead + it] : -1;
            }
            __syncthreads();
            const int kc = L.item;
            __syncthreads();
            if (kc < 0) break;
            fix_velocity(A, J, cand, L, kc);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(head + 2, 1) == (int)gridDim.x - 1) {
        for (int j = 0; j < njobs; ++j) {
            int* f = get(j).flag;
            f[0] = 0;
            f[1] = 0;
        }
        __threadfence();
        head[2] = 0;
    }
}

struct FixOne {
    MergeJob job;
    sst_candidate* cand;
};

__global__ __launch_bounds__(kAux) void k_fixup(const StackArgs A, const FixOne F) {
    const KArgs Ap = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
    fix_loop(1, [&](int, KArgs* a = nullptr, sst_candidate** c = nullptr) -> const MergeJob& {
        if (a) *a = Ap;
        if (c) *c = F.cand;
        return F.job;
    });
}

__global__ __launch_bounds__(kAux) void k_fixup_batch(const MergeBatch B) {
    fix_loop(B.np, [&](int j, KArgs* a = nullptr, sst_candidate** c = nullptr) -> const MergeJob& {
        if (a) *a = B.jobs[j].args;
        if (c) *c = B.cand[j];
        return B.jobs[j];
    });
}

hipError_t launch_fixup(const StackArgs& a, const MergeJob& job, void* cand, int32_t*, int groups, hipStream_t s) {
    FixOne f{job, static_cast<sst_candidate*>(cand)};
    hipLaunchKernelGGL(k_fixup, dim3((unsigned)groups), dim3(kAux), 0, s, a, f);
    return hipGetLastError();
}

hipError_t launch_fixup_batch(const MergeBatch& b, int groups, hipStream_t s) {
    if (b.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fixup_batch, dim3((unsigned)groups), dim3(kAux), 0, s, b);
    return hipGetLastError();
}

// ------------------------------------------------------------- launchers
hipError_t launch_stats(const void* frames, int dtype, const float* scale, int n, int h, int w, double* part,
                        int nchunk, double* b, double* s2, float* b32, double* P, double* Pb, double* stats_dev,
                        hipStream_t s) {
    const long long npx = (long long)h * w;
    const dim3 grid(nchunk, n);
    if (dtype == SST_BF16)
        hipLaunchKernelGGL(k_stats_partial<SST_BF16>, grid, dim3(kAux), 0, s, frames, scale, npx, nchunk, part);
    else if (dtype == SST_F16)
        hipLaunchKernelGGL(k_stats_partial<SST_F16>, grid, dim3(kAux), 0, s, frames, scale, npx, nchunk, part);
    else
        hipLaunchKernelGGL(k_stats_partial<SST_F32>, grid, dim3(kAux), 0, s, frames, scale, npx, nchunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kAux), 0, s, part, nchunk, n, npx, b, s2, b32, P, Pb,
                       stats_dev);
    return hipGetLastError();
}

hipError_t launch_quantize(const float* frames, int n, int h, int w, int dtype, const float* offset, float* part,
                           int nchunk, float* scale, void* q, hipStream_t s) {
    const long long npx = (long long)h * w;
    hipLaunchKernelGGL(k_absmax_partial, dim3(nchunk, n), dim3(kAux), 0, s, frames, npx, offset, nchunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kAux), 0, s, part, nchunk, n, scale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 grid((unsigned)((npx + kAux - 1) / kAux), n);
    uint16_t* qb = static_cast<uint16_t*>(q);
    if (dtype == SST_BF16)
        hipLaunchKernelGGL(k_quantize<SST_BF16>, grid, dim3(kAux), 0, s, frames, npx, offset, scale, qb);
    else
        hipLaunchKernelGGL(k_quantize<SST_F16>, grid, dim3(kAux), 0, s, frames, npx, offset, scale, qb);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
    const long long chunks = (long long)(a.Hp / 4) * a.Wp;
    const dim3 grid((unsigned)((chunks + kAux - 1) / kAux), a.n);
    if (a.half && a.dtype == SST_F16)
        hipLaunchKernelGGL(k_prep_half, grid, dim3(kAux), 0, s, a);
    else if (a.dtype == SST_BF16)
        hipLaunchKernelGGL(k_prep<SST_BF16>, grid, dim3(kAux), 0, s, a);
    else if (a.dtype == SST_F16)
        hipLaunchKernelGGL(k_prep<SST_F16>, grid, dim3(kAux), 0, s, a);
    else
        hipLaunchKernelGGL(k_prep<SST_F32>, grid, dim3(kAux), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cov(const int* D, int ld, int n, int nv, int size, int* I, hipStream_t s) {
    hipLaunchKernelGGL(k_cov, dim3((size + kAux - 1) / kAux, nv), dim3(kAux), 0, s, D, ld, n, size, I);
    return hipGetLastError();
}

template <int SH>
void launch_stack_shape(const StackArgs& a, bool detect, bool staged, dim3 grid, hipStream_t s) {
    const dim3 block(shape_waves(SH) * kWave);
    if constexpr (SH == 2) {
        if (detect && staged && !a.half && a.redo) {
            // two passes: the search without candidates at four workgroups
            // per CU, then in full the items it listed
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(kAux), 0, s, a.redo, kRedoHead);
            hipLaunchKernelGGL((k_stack<true, true, SH, false, true>), grid, block, 0, s, a);
            const dim3 chunks((grid.x + kCompactChunk - 1) / kCompactChunk);
            hipLaunchKernelGGL(k_redo_count, chunks, dim3(kCompactThreads), 0, s, a.redo, (int)grid.x);
            hipLaunchKernelGGL(k_redo_list, chunks, dim3(kCompactThreads), 0, s, a.redo, (int)grid.x);
            hipLaunchKernelGGL(k_stack_redo<SH>, dim3((grid.x + kRedoRuns - 1) / kRedoRuns * kRedoRuns), block, 0,
                               s, a, (int)grid.x);
            return;
        }
    }
    if (detect) {
        if (staged && a.half)
            hipLaunchKernelGGL((k_stack<true, true, SH, true>), grid, block, 0, s, a);
        else if (staged)
            hipLaunchKernelGGL((k_stack<true, true, SH, false>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_stack<true, false, SH, false>), grid, block, 0, s, a);
    } else {
        if (staged)
            hipLaunchKernelGGL((k_stack<false, true, SH, false>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_stack<false, false, SH, false>), grid, block, 0, s, a);
    }
}

hipError_t launch_stack(const StackArgs& a, bool detect, bool staged, int shape, hipStream_t s) {
    const long long groups = (long long)a.tiles_x * a.tiles_y * shape_items_per_tile(shape) * a.nvbx * a.nvby;
    const dim3 grid((unsigned)groups);
    static_assert(kNShapes == 3, "one instantiation per shape");
    if (shape == 2)
        launch_stack_shape<2>(a, detect, staged, grid, s);
    else if (shape == 1)
        launch_stack_shape<1>(a, detect, staged, grid, s);
    else
        launch_stack_shape<0>(a, detect, staged, grid, s);
    return hipGetLastError();
}

// rec[kRecScale] = bits of scale[rec[4]] in every record
__global__ __launch_bounds__(kAux) void k_rec_scale(int* ord, long long ord_stride, int nrec, long long total,
                                                     int rec, const float* __restrict__ scale) {
    const long long t = (long long)blockIdx.x * kAux + threadIdx.x;
    if (t >= total) return;
    const long long b = t / nrec, k = t - b * nrec;
    int* r = ord + b * ord_stride + kCountInts + k * rec;
    r[kRecScale] = __float_as_int(scale[r[4]]);
}

hipError_t launch_rec_scale(int* ord, int nblk, long long ord_stride, int nrec, int rec, const float* scale,
                            hipStream_t s) {
    const long long total = (long long)nblk * nrec;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rec_scale, dim3((unsigned)((total + kAux - 1) / kAux)), dim3(kAux), 0, s, ord, ord_stride,
                       nrec, total, rec, scale);
    return hipGetLastError();
}

hipError_t launch_stack_batch(const BatchArgs& b, int groups, int shape, hipStream_t s) {
    if (groups <= 0) return hipSuccess;
    if (shape == 2)
        hipLaunchKernelGGL(k_stack_batch<2>, dim3((unsigned)groups), dim3(shape_waves(2) * kWave), 0, s, b);
    else if (shape == 1)
        hipLaunchKernelGGL(k_stack_batch<1>, dim3((unsigned)groups), dim3(shape_waves(1) * kWave), 0, s, b);
    else
        hipLaunchKernelGGL(k_stack_batch<0>, dim3((unsigned)groups), dim3(shape_waves(0) * kWave), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int* p, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((count + kAux - 1) / kAux)), dim3(kAux), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_merge(const int32_t* tcount, const Entry* ent, int nslot, int kt, int k_max, int nvx, int w,
                        int k_first, int nk, void* cand, int32_t* count, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_merge, dim3(nk), dim3(kAux), 0, s, tcount, ent, nslot, kt, k_max, nvx, w, k_first,
                       static_cast<sst_candidate*>(cand), count, flag);
    return hipGetLastError();
}

}  // namespace sst
