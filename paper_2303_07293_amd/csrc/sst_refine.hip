// Differentiable sub-pixel refinement of detections, written for gfx950.
//
// A detection of the search is an integer pixel and a trial velocity on the
// grid (paper Sec. 2.1).  Refinement treats theta = (x0, y0, vx, vy) as
// continuous: a C x C cutout is stacked with bilinear sampling along the
// linear track, G_i = F_i - b_i zero outside the frame,
//     Cut(u, v) = sum_i bilin(G_i; x0 + u + vx dt_i, y0 + v + vy dt_i),
// and the objective is the PSF-weighted S/N
//     SN = sum_{u,v} w(u,v) Cut(u,v) / sqrt(sum w^2 * sum_i s2_i)
// whose normaliser does not depend on theta.  Its exact (piecewise)
// gradient is the hand-written adjoint below; gradient ascent runs inside
// the kernel.
//
// Layout: the offsets u, v are integers, so for frame i every sample of the
// cutout has the same fractional offset (fx, fy) and the cutout touches the
// (C+1) x (C+1) pixel window anchored at floor(x0 + vx dt_i) - R.  Each
// window pixel enters the weighted sum through the four PSF weights of the
// cutout samples that touch it, so numerator and gradient are single
// weighted sums over the window: one gather per window pixel and frame.
// One workgroup per candidate runs all ascent steps; nothing crosses
// workgroups.
#include "sst_internal.h"

#include <climits>

namespace sst {

constexpr int kRefThreads = 256;
constexpr int kRefMaxC = 63;
constexpr int kRefW = kRefMaxC + 2;  // weight table side: cutout plus a zero border

__device__ __forceinline__ float block_sum5(float (&v)[5], float* sh) {
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k) sh[k * 4 + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = (sh[k * 4 + 0] + sh[k * 4 + 1]) + (sh[k * 4 + 2] + sh[k * 4 + 3]);
    __syncthreads();
    return v[0];
}

// Window pixels per thread held in registers (KPER > 0: cutouts with
// (C + 1)^2 <= KPER * kRefThreads): each thread's pixels, their window
// coordinates and their four PSF weights do not change over frames and
// steps, so they are computed once.  KPER = 0: the general loop, which
// recomputes them per frame.  Both visit a thread's pixels in the same
// order with the same arithmetic.
constexpr int kRefPer = 5;

template <int DT, int KPER>
__global__ __launch_bounds__(kRefThreads) void k_refine(const RefineArgs A) {
    static_assert(kRefThreads == 4 * kWave, "four waves per candidate");
    __shared__ float wt[kRefW * kRefW];  // wt[(v + R + 1) * (C + 2) + (u + R + 1)], zero border
    __shared__ float sh[20];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int C = A.cutout, R = C / 2, CW = C + 2, nel = (C + 1) * (C + 1);
    const float inv2s2 = A.inv2s2;
    for (int e = tid; e < CW * CW; e += kRefThreads) {
        const int r = e / CW, q = e - r * CW;
        float v = 0.f;
        if (r >= 1 && r <= C && q >= 1 && q <= C) {
            const float du = (float)(q - 1 - R), dv = (float)(r - 1 - R);
            v = expf(-(du * du + dv * dv) * inv2s2);
        }
        wt[e] = v;
    }
    // normaliser: sum of PSF weights squared (float64 from the host) times
    // the total frame variance P[n]
    const double vtot = A.P[A.n];
    const float inv_norm = vtot > 0.0 ? rsqrtf((float)(A.sw2 * vtot)) : 0.f;
    __syncthreads();

    int er[KPER > 0 ? KPER : 1], eq[KPER > 0 ? KPER : 1];
    float w00[KPER > 0 ? KPER : 1], w01[KPER > 0 ? KPER : 1], w10[KPER > 0 ? KPER : 1], w11[KPER > 0 ? KPER : 1];
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
        const int e = tid + k * kRefThreads;
        const int r = e < nel ? e / (C + 1) : 0, q = e < nel ? e - r * (C + 1) : 0;
        // pixels past the window get an empty row, which fails the bounds test
        er[k] = e < nel ? r : INT_MIN / 2;
        eq[k] = q;
        w00[k] = wt[(r + 1) * CW + q + 1];
        w01[k] = wt[(r + 1) * CW + q];
        w10[k] = wt[r * CW + q + 1];
        w11[k] = wt[r * CW + q];
    }

    float th[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) th[k] = A.params[(long long)c * 4 + k];
    float sn = 0.f, g[4] = {0.f, 0.f, 0.f, 0.f};
    for (int step = 0; step <= A.steps; ++step) {
        float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // numerator, d/dx0, d/dy0, d/dvx, d/dvy
        for (int i = 0; i < A.n; ++i) {
            const float dt = A.dt[i];
            const float X0 = th[0] + th[2] * dt, Y0 = th[1] + th[3] * dt;
            const float ax = floorf(X0), ay = floorf(Y0);
            const float fx = X0 - ax, fy = Y0 - ay;
            const float k00 = (1.f - fx) * (1.f - fy), k01 = fx * (1.f - fy);
            const float k10 = (1.f - fx) * fy, k11 = fx * fy;
            // the window's origin in frame pixels (clamped far outside the
            // frame: such samples are all zero)
            const int ix = (int)fminf(fmaxf(ax, -1e8f), 1e8f) - R;
            const int iy = (int)fminf(fmaxf(ay, -1e8f), 1e8f) - R;
            const float sc = DT == SST_F32 ? 1.f : A.scale[i];
            const float bi = A.b32[i];
            const long long fbase = (long long)i * A.h * A.w;
            float tx = 0.f, ty = 0.f;
            auto one = [&](int r, int q, float p00, float p01, float p10, float p11) __attribute__((always_inline)) {
                const int px = ix + q, py = iy + r;
                if (px < 0 || px >= A.w || py < 0 || py >= A.h) return;
                const float G = frame_value<DT>(A.frames, fbase + (long long)py * A.w + px, sc) - bi;
                acc[0] += G * (((k00 * p00 + k01 * p01) + k10 * p10) + k11 * p11);
                tx += G * ((1.f - fy) * (p01 - p00) + fy * (p11 - p10));
                ty += G * ((1.f - fx) * (p10 - p00) + fx * (p11 - p01));
            };
            if constexpr (KPER > 0) {
#pragma unroll
                for (int k = 0; k < KPER; ++k) one(er[k], eq[k], w00[k], w01[k], w10[k], w11[k]);
            } else {
                for (int e = tid; e < nel; e += kRefThreads) {
                    const int r = e / (C + 1), q = e - r * (C + 1);
                    one(r, q, wt[(r + 1) * CW + q + 1], wt[(r + 1) * CW + q], wt[r * CW + q + 1], wt[r * CW + q]);
                }
            }
            acc[1] += tx;
            acc[2] += ty;
            acc[3] += dt * tx;
            acc[4] += dt * ty;
        }
        block_sum5(acc, sh);
        sn = acc[0] * inv_norm;
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = acc[k + 1] * inv_norm;
        if (step < A.steps)
#pragma unroll
            for (int k = 0; k < 4; ++k) th[k] += A.lr * g[k];
    }
    if (tid == 0) {
        A.snr[c] = sn;
#pragma unroll
        for (int k = 0; k < 4; ++k) A.params[(long long)c * 4 + k] = th[k];
        if (A.grad)
#pragma unroll
            for (int k = 0; k < 4; ++k) A.grad[(long long)c * 4 + k] = g[k];
    }
}

template <int KPER>
void launch_refine_per(const RefineArgs& a, hipStream_t s) {
    if (a.dtype == SST_BF16)
        hipLaunchKernelGGL((k_refine<SST_BF16, KPER>), dim3(a.nc), dim3(kRefThreads), 0, s, a);
    else if (a.dtype == SST_F16)
        hipLaunchKernelGGL((k_refine<SST_F16, KPER>), dim3(a.nc), dim3(kRefThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_refine<SST_F32, KPER>), dim3(a.nc), dim3(kRefThreads), 0, s, a);
}

hipError_t launch_refine(const RefineArgs& a, hipStream_t s) {
    if (a.nc == 0) return hipSuccess;
    if ((a.cutout + 1) * (a.cutout + 1) <= kRefPer * kRefThreads)
        launch_refine_per<kRefPer>(a, s);
    else
        launch_refine_per<0>(a, s);
    return hipGetLastError();
}

}  // namespace sst
