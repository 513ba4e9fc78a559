// HIP kernels of the steps the paper runs just before the search, written
// for gfx950.  All three are memory-bound streaming kernels with coalesced
// row-major access; none is on the search's hot path.
//
//   k_median_sub  static-source removal (paper Sec. 2.1: the median
//                 combination of a group's frames is removed from each
//                 frame): out_i(p) = F_i(p) - median_j F_j(p)
//   k_coadd       summing every `group` consecutive frames (Sec. 2.1 and
//                 Sec. 2.2: co-added frames for the slow-mover search)
//   k_bin2x2      2x2 binning (Sec. 2.3: binned frames for the fast-mover
//                 search): each output pixel is the sum of a 2x2 block
#include "sst_internal.h"
#include "../../include/sst.h"

namespace sst {

constexpr int kPrepThreads = 256;

// ---------------------------------------------------------------- median
// float32 <-> unsigned key with the same order (finite values; -0 sorts just
// below +0, which compare equal as numbers)
__device__ __forceinline__ unsigned order_key(float v) {
    const unsigned u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(unsigned k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// One wave per 64 pixels; the n samples of each lane's pixel are staged in
// LDS as order keys (key[j * 64 + lane]).  The j-th smallest key is the
// largest r with #(key < r) <= j, built bit by bit from the top (the
// predicate is monotone in r): 32 counting passes over the n keys.
__global__ __launch_bounds__(kWave) void k_median_sub(const float* __restrict__ F, int n, long long npx,
                                                         float* __restrict__ out, float* __restrict__ med_out) {
    extern __shared__ unsigned keys[];
    const int lane = threadIdx.x;
    const long long p = (long long)blockIdx.x * kWave + lane;
    const bool in = p < npx;
    for (int j = 0; j < n; ++j) keys[j * kWave + lane] = order_key(in ? F[(long long)j * npx + p] : 0.f);
    auto select = [&](int j) {
        unsigned r = 0;
        for (int b = 31; b >= 0; --b) {
            const unsigned trial = r | (1u << b);
            int below = 0;
            for (int i = 0; i < n; ++i) below += keys[i * kWave + lane] < trial;
            if (below <= j) r = trial;
        }
        return r;
    };
    const int k = (n - 1) / 2;
    const unsigned lo = select(k);
    float med = key_value(lo);
    if ((n & 1) == 0) {
        // the next order statistic: lo again if it repeats, else the
        // smallest key above lo
        int le = 0;
        unsigned nxt = 0xFFFFFFFFu;
        for (int i = 0; i < n; ++i) {
            const unsigned kk = keys[i * kWave + lane];
            le += kk <= lo;
            if (kk > lo && kk < nxt) nxt = kk;
        }
        const unsigned hi = le >= k + 2 ? lo : nxt;
        med = (key_value(lo) + key_value(hi)) * 0.5f;
    }
    if (!in) return;
    for (int j = 0; j < n; ++j) out[(long long)j * npx + p] = key_value(keys[j * kWave + lane]) - med;
    if (med_out) med_out[p] = med;
}

// Register form for n <= kMedRegs (group sizes of tens of frames): each
// lane holds its pixel's keys in registers, so the counting passes touch no
// memory.  Keys past n are the largest key, which is never below a trial
// value, so they are never counted and never chosen.  Same selection, so
// the same median and outputs bit for bit as the LDS form.
constexpr int kMedRegs = 64;

__global__ __launch_bounds__(kPrepThreads) void k_median_sub_reg(const float* __restrict__ F, int n, long long npx,
                                                                    float* __restrict__ out,
                                                                    float* __restrict__ med_out) {
    const long long p = (long long)blockIdx.x * kPrepThreads + threadIdx.x;
    if (p >= npx) return;
    unsigned key[kMedRegs];
#pragma unroll
    for (int j = 0; j < kMedRegs; ++j) key[j] = j < n ? order_key(F[(long long)j * npx + p]) : 0xFFFFFFFFu;
    // every order statistic lies in [kmin, kmax], so it shares their common
    // leading bits: the bit-by-bit search starts below them
    unsigned kmin = key[0], kmax = key[0];
#pragma unroll
    for (int j = 1; j < kMedRegs; ++j)
        if (j < n) {
            kmin = min(kmin, key[j]);
            kmax = max(kmax, key[j]);
        }
    const int top = 31 - __clz((int)(kmin ^ kmax));  // highest differing bit, -1 if none
    const unsigned prefix = top < 0 ? kmin : kmin & ~((2u << top) - 1u);
    auto select = [&](int j) {
        unsigned r = prefix;
#pragma unroll 1
        for (int b = top; b >= 0; --b) {
            const unsigned trial = r | (1u << b);
            int below = 0;
#pragma unroll
            for (int i = 0; i < kMedRegs; ++i) below += key[i] < trial;
            if (below <= j) r = trial;
        }
        return r;
    };
    const int k = (n - 1) / 2;
    const unsigned lo = select(k);
    float med = key_value(lo);
    if ((n & 1) == 0) {
        int le = 0;
        unsigned nxt = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < kMedRegs; ++i) {
            le += key[i] <= lo;
            if (key[i] > lo && key[i] < nxt) nxt = key[i];
        }
        const unsigned hi = le >= k + 2 ? lo : nxt;
        med = (key_value(lo) + key_value(hi)) * 0.5f;
    }
#pragma unroll
    for (int j = 0; j < kMedRegs; ++j)
        if (j < n) out[(long long)j * npx + p] = key_value(key[j]) - med;
    if (med_out) med_out[p] = med;
}

// ---------------------------------------------------------------- co-add
// out[g][p] = sum over j < group, ascending, of F[g * group + j][p]
__global__ __launch_bounds__(kPrepThreads) void k_coadd(const float* __restrict__ F, long long npx, int group,
                                                           float* __restrict__ out) {
    const int g = blockIdx.y;
    const long long p = (long long)blockIdx.x * kPrepThreads + threadIdx.x;
    if (p >= npx) return;
    const float* f = F + (long long)g * group * npx + p;
    float s = 0.f;
    for (int j = 0; j < group; ++j) s += f[(long long)j * npx];
    out[(long long)g * npx + p] = s;
}

// ---------------------------------------------------------------- binning
// out[i][y][x] = (F[2y][2x] + F[2y][2x+1]) + (F[2y+1][2x] + F[2y+1][2x+1]);
// an odd last row or column is dropped
__global__ __launch_bounds__(kPrepThreads) void k_bin2x2(const float* __restrict__ F, int h, int w,
                                                            float* __restrict__ out, int ho, int wo) {
    const int i = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * kPrepThreads + threadIdx.x;
    if (x >= wo) return;
    const float* r0 = F + ((long long)i * h + 2 * y) * w + 2 * x;
    const float* r1 = r0 + w;
    out[((long long)i * ho + y) * wo + x] = (r0[0] + r0[1]) + (r1[0] + r1[1]);
}

hipError_t launch_median_sub(const float* F, int n, int h, int w, float* out, float* med, hipStream_t s) {
    const long long npx = (long long)h * w;
    if (n <= kMedRegs) {
        const unsigned blocks = (unsigned)((npx + kPrepThreads - 1) / kPrepThreads);
        hipLaunchKernelGGL(k_median_sub_reg, dim3(blocks), dim3(kPrepThreads), 0, s, F, n, npx, out, med);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((npx + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_median_sub, dim3(blocks), dim3(kWave), (size_t)n * kWave * sizeof(unsigned), s, F, n, npx,
                       out, med);
    return hipGetLastError();
}

hipError_t launch_coadd(const float* F, int h, int w, int group, int ng, float* out, hipStream_t s) {
    const long long npx = (long long)h * w;
    hipLaunchKernelGGL(k_coadd, dim3((unsigned)((npx + kPrepThreads - 1) / kPrepThreads), ng), dim3(kPrepThreads),
                       0, s, F, npx, group, out);
    return hipGetLastError();
}

hipError_t launch_bin2x2(const float* F, int n, int h, int w, float* out, hipStream_t s) {
    const int ho = h / 2, wo = w / 2;
    hipLaunchKernelGGL(k_bin2x2, dim3((wo + kPrepThreads - 1) / kPrepThreads, ho, n), dim3(kPrepThreads), 0, s, F,
                       h, w, out, ho, wo);
    return hipGetLastError();
}

}  // namespace sst
