// gfx950 kernels of the tracking pose solve and of the canonical pointmap
// fusion that follows it (MASt3R-SLAM, Sec. 3.3).
//
// Robustly weighted Gauss-Newton, the weights recomputed every iteration
// (Eq. gauss_newton), for the Sim(3) pose T_kf that maps frame points X^f_f into the
// keyframe, over the matches of the keyframe's pixels found by the matcher.
// One launch per iteration:
//
//   step    every workgroup first sums the previous iteration's partials in
//           fp64 in a fixed order, solves the 7x7 system by Cholesky and
//           applies T <- Exp(tau) o T (Eq. 1, left plus on Sim(3)) in fp64:
//           the same arithmetic in every workgroup, so every workgroup holds
//           the same new pose, and workgroup 0 records it.  Then one lane per
//           match n: x = T Xf[m] with m = idx[n]; ray residual psi(x) -
//           psi(Xk[n]) (Eq. track_ray) and distance residual |x| - |Xk[n]|
//           (the small-weight distance term); Jacobians w.r.t. a left
//           perturbation (Supp. A); weights q / sigma^2 (match confidence q =
//           sqrt(Qf[m] Qk[n]) gated at q_min, Sec. 3.3) times the Huber weight
//           of the whitened block norm; one fp32 partial of J^T W J (upper
//           triangle), J^T W r, robust cost and count per workgroup.
//   final   one workgroup: the last partials summed (cost and count at the
//           final pose), the fp32 pose and the statistics written.
//
// The partials and the fp64 pose are double-buffered by iteration parity, so
// a launch reads what the previous launch wrote and no workgroup overwrites
// what another still reads; kernel boundaries order every hand-off (no
// device-scope fence: on this part a device-scope release writes back the
// XCD's L2).  Launches are stream-ordered with no host synchronisation, so
// the whole solve can be captured into a graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m3s_internal.h"
#include "m3s_sim3.h"

namespace m3s {

namespace {

constexpr int kThreads = 256;
constexpr int kVals = kPoseVals;
constexpr int kStride = 40;         // floats per block partial
constexpr int kMaxBlocks = 2048;

// Workspace layout (bytes): poses, statistics, counters, then the partials.
constexpr size_t kOffT = 0;         // double[2][12]: pose by iteration parity
constexpr size_t kOffStat = 192;    // double[2]: last step norm, reserved
constexpr size_t kOffCnt = 224;     // int32[2]: reserved, solved iterations
constexpr size_t kOffPart = 256;    // float[2][nblocks * kStride]: partials by iteration parity

struct TrackArgs {
    int N;
    const float* Xk;
    const float* Xf;
    const int32_t* idx;
    const uint8_t* valid;
    const float* Qf;
    const float* Qk;
    double q_min;
    float q_minf;
    RobustWeights rw;
    double* T64;            // [2][12]
    double* stat;
    int32_t* counter;       // [0] reserved, [1] solved iterations
    int32_t* solved;
    float* partials;        // [2][nb * kStride]
    int nb;
    float* T_out;
    float* info;
};

__global__ void __launch_bounds__(64) track_init_kernel(const float* __restrict__ T_in, double* __restrict__ T64,
                                                        int32_t* __restrict__ cnt, double* __restrict__ stat) {
    const int i = threadIdx.x;
    if (i < 12) T64[i] = (double)T_in[i];
    if (i < 2) { cnt[i] = 0; stat[i] = 0.0; }
}

// Solve H tau = -g (7x7 SPD) and apply T <- Exp(tau) o T.  Returns false
// (pose unchanged) when H is not positive definite.
__device__ bool solve_and_update(const double* sum, double* T, double* step_norm) {
    // Cholesky by rows; each pivot's reciprocal serves its column and both
    // substitutions (one fp64 division per pivot).
    double L[7][7], inv[7];
    for (int r = 0; r < 7; ++r)
        for (int c = 0; c < 7; ++c) L[r][c] = 0.0;
    for (int r = 0; r < 7; ++r) {
        for (int c = 0; c <= r; ++c) {
            double s = sum[upper_index(c, r)];
            for (int q = 0; q < c; ++q) s -= L[r][q] * L[c][q];
            if (r == c) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                L[r][r] = sqrt(s);
                inv[r] = 1.0 / L[r][r];
            } else {
                L[r][c] = s * inv[c];
            }
        }
    }
    double y[7], tau[7];
    for (int r = 0; r < 7; ++r) {
        double s = -sum[28 + r];
        for (int q = 0; q < r; ++q) s -= L[r][q] * y[q];
        y[r] = s * inv[r];
    }
    for (int r = 6; r >= 0; --r) {
        double s = y[r];
        for (int q = r + 1; q < 7; ++q) s -= L[q][r] * tau[q];
        tau[r] = s * inv[r];
    }
    double E[12], Tn[12];
    sim3_exp(tau, E);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c)
            Tn[4 * r + c] = E[4 * r] * T[c] + E[4 * r + 1] * T[4 + c] + E[4 * r + 2] * T[8 + c] +
                            (c == 3 ? E[4 * r + 3] : 0.0);
    for (int j = 0; j < 12; ++j) T[j] = Tn[j];
    double tn = 0.0;
    for (int j = 0; j < 7; ++j) tn += tau[j] * tau[j];
    *step_norm = sqrt(tn);
    return true;
}

// Normal equations of the matches of this workgroup at the current pose: one
// fp32 partial of kVals values per workgroup.
// Matches per lane and step of the accumulation: their reads are issued
// together before the arithmetic.
constexpr int kMatchesPerLane = 4;

__global__ void __launch_bounds__(kThreads) track_step_kernel(TrackArgs A, int it) {
    __shared__ float red[kThreads / 64][kVals];
    __shared__ double sum[kVals];
    __shared__ double part[kThreads / kVals * kVals];
    __shared__ double Tn[12];
    // Pose of the previous iteration (parity buffer); iteration 0 starts from
    // the initial pose in buffer 0.
    const double* Tprev = A.T64 + (it > 0 ? 12 * ((it + 1) & 1) : 0);
    if (it > 0) {
        // Iteration it - 1's system: the same fixed-order sum and solve in
        // every workgroup.
        sum_partials<kThreads>(A.partials + (size_t)((it + 1) & 1) * A.nb * kStride, A.nb, kStride, part, sum);
        if (threadIdx.x == 0) {
            double Tl[12], step;
            for (int j = 0; j < 12; ++j) Tl[j] = Tprev[j];
            const bool ok = solve_and_update(sum, Tl, &step);
            for (int j = 0; j < 12; ++j) Tn[j] = Tl[j];
            if (blockIdx.x == 0) {
                double* Tout = A.T64 + 12 * (it & 1);
                for (int j = 0; j < 12; ++j) Tout[j] = Tl[j];
                if (ok) {
                    A.solved[0] += 1;
                    A.stat[0] = step;
                }
            }
        }
    } else if (threadIdx.x < 12) {
        Tn[threadIdx.x] = Tprev[threadIdx.x];
    }
    __syncthreads();
    float T[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) T[i] = (float)Tn[i];
    float acc[kVals];
#pragma unroll
    for (int i = 0; i < kVals; ++i) acc[i] = 0.f;

    constexpr int kStep = kThreads * kMatchesPerLane;
    for (int base = blockIdx.x * kStep + threadIdx.x; base < A.N; base += gridDim.x * kStep) {
        int nn[kMatchesPerLane], mm[kMatchesPerLane];
        bool ok[kMatchesPerLane];
#pragma unroll
        for (int u = 0; u < kMatchesPerLane; ++u) {
            nn[u] = base + u * kThreads;
            ok[u] = nn[u] < A.N && A.valid[nn[u]];
            mm[u] = ok[u] ? A.idx[nn[u]] : 0;
            ok[u] = ok[u] && mm[u] >= 0 && mm[u] < A.N;
        }
        float qf[kMatchesPerLane], qk[kMatchesPerLane], xf[kMatchesPerLane][3], xk[kMatchesPerLane][3];
#pragma unroll
        for (int u = 0; u < kMatchesPerLane; ++u) {
            const int m = ok[u] ? mm[u] : 0, n = ok[u] ? nn[u] : 0;
            qf[u] = A.Qf[m]; qk[u] = A.Qk[n];
#pragma unroll
            for (int j = 0; j < 3; ++j) { xf[u][j] = A.Xf[3 * m + j]; xk[u][j] = A.Xk[3 * n + j]; }
        }
#pragma unroll
        for (int u = 0; u < kMatchesPerLane; ++u) {
            float q;
            if (ok[u] && confidence_gate(qf[u], qk[u], A.q_min, A.q_minf, q))
                accumulate_match(T, xf[u][0], xf[u][1], xf[u][2], xk[u][0], xk[u][1], xk[u][2], q, A.rw, acc);
        }
    }

    // Block partial: wave sums, then the four waves through LDS.
#pragma unroll
    for (int i = 0; i < kVals; ++i) acc[i] = wave_sum(acc[i]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < kVals; ++i) red[threadIdx.x >> 6][i] = acc[i];
    }
    __syncthreads();
    if (threadIdx.x < kVals) {
        float v = 0.f;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
        A.partials[((size_t)(it & 1) * A.nb + blockIdx.x) * kStride + threadIdx.x] = v;
    }
}

// One workgroup: the last iteration's partials summed (cost and count at the
// final pose), the fp32 pose and the statistics written.
__global__ void __launch_bounds__(kThreads) track_final_kernel(TrackArgs A, int it) {
    __shared__ double sum[kVals];
    __shared__ double part[kThreads / kVals * kVals];
    sum_partials<kThreads>(A.partials + (size_t)(it & 1) * A.nb * kStride, A.nb, kStride, part, sum);
    if (threadIdx.x != 0) return;
    const double* T = A.T64 + 12 * (it & 1);
    for (int j = 0; j < 12; ++j) A.T_out[j] = (float)T[j];
    if (A.info) {
        A.info[0] = (float)sum[35];
        A.info[1] = (float)sum[36];
        A.info[2] = (float)A.solved[0];
        A.info[3] = (float)A.stat[0];
    }
}

// Canonical pointmap update (Sec. 3.3, Eq. 8), per keyframe pixel n:
//   Xc[n] <- (Cc[n] Xc[n] + C[n] (T X[n])) / (Cc[n] + C[n]),  Cc[n] <- Cc[n] + C[n];
// a pixel whose summed confidence is not positive keeps its point.  VEC
// pixels per lane: with VEC = 4 every array is read and written as float4
// (3 per point quad, 1 per confidence quad); VEC = 1 handles any alignment
// and the tail.
__device__ __forceinline__ void fuse_one(const float* T, float& x0, float& x1, float& x2, float& cc, float X0, float X1,
                                         float X2, float c) {
    const float t0 = T[0] * X0 + T[1] * X1 + T[2] * X2 + T[3];
    const float t1 = T[4] * X0 + T[5] * X1 + T[6] * X2 + T[7];
    const float t2 = T[8] * X0 + T[9] * X1 + T[10] * X2 + T[11];
    const float cs = cc + c;
    if (cs > 0.f) {
        const float inv = 1.f / cs;
        x0 = (cc * x0 + c * t0) * inv;
        x1 = (cc * x1 + c * t1) * inv;
        x2 = (cc * x2 + c * t2) * inv;
    }
    cc = cs;
}

template <int VEC>
__global__ void __launch_bounds__(256) fuse_kernel(int N, int first, const float* __restrict__ Tg, float* __restrict__ Xc,
                                                   float* __restrict__ Cc, const float* __restrict__ X,
                                                   const float* __restrict__ C) {
    float T[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) T[i] = Tg[i];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (VEC == 4) {
        const long n0 = first + 4 * g;
        if (n0 + 4 > N) return;
        float4* xc4 = reinterpret_cast<float4*>(Xc + 3 * n0);
        const float4* x4 = reinterpret_cast<const float4*>(X + 3 * n0);
        float4 a = xc4[0], b = xc4[1], d = xc4[2];
        const float4 p = x4[0], q = x4[1], r = x4[2];
        float4 cc = *reinterpret_cast<const float4*>(Cc + n0);
        const float4 c = *reinterpret_cast<const float4*>(C + n0);
        fuse_one(T, a.x, a.y, a.z, cc.x, p.x, p.y, p.z, c.x);
        fuse_one(T, a.w, b.x, b.y, cc.y, p.w, q.x, q.y, c.y);
        fuse_one(T, b.z, b.w, d.x, cc.z, q.z, q.w, r.x, c.z);
        fuse_one(T, d.y, d.z, d.w, cc.w, r.y, r.z, r.w, c.w);
        xc4[0] = a; xc4[1] = b; xc4[2] = d;
        *reinterpret_cast<float4*>(Cc + n0) = cc;
    } else {
        const long n = first + g;
        if (n >= N) return;
        float x0 = Xc[3 * n], x1 = Xc[3 * n + 1], x2 = Xc[3 * n + 2], cc = Cc[n];
        fuse_one(T, x0, x1, x2, cc, X[3 * n], X[3 * n + 1], X[3 * n + 2], C[n]);
        Xc[3 * n] = x0; Xc[3 * n + 1] = x1; Xc[3 * n + 2] = x2;
        Cc[n] = cc;
    }
}

}  // namespace

int track_blocks(int N) {
    const int nb = (N + kThreads * kMatchesPerLane - 1) / (kThreads * kMatchesPerLane);
    return nb < 1 ? 1 : (nb > kMaxBlocks ? kMaxBlocks : nb);
}

size_t track_workspace_bytes(int N) { return kOffPart + 2 * (size_t)track_blocks(N) * kStride * sizeof(float); }

hipError_t launch_track(int N, const float* Xk, const float* Xf, const int32_t* idx, const uint8_t* valid,
                        const float* Qf, const float* Qk, float q_min, float sigma_ray, float sigma_dist, float huber,
                        int iters, float* T, float* info, void* ws, hipStream_t s) {
    char* w = reinterpret_cast<char*>(ws);
    TrackArgs A;
    A.N = N;
    A.Xk = Xk; A.Xf = Xf; A.idx = idx; A.valid = valid; A.Qf = Qf; A.Qk = Qk;
    A.q_min = (double)q_min;
    A.q_minf = q_min;
    // An infinite sigma drops its residual from the system and the cost.
    A.rw = robust_weights(sigma_ray, sigma_dist, huber);
    A.T64 = reinterpret_cast<double*>(w + kOffT);
    A.stat = reinterpret_cast<double*>(w + kOffStat);
    A.counter = reinterpret_cast<int32_t*>(w + kOffCnt);
    A.solved = A.counter + 1;
    A.partials = reinterpret_cast<float*>(w + kOffPart);
    A.T_out = T;
    A.info = info;
    const int nb = track_blocks(N);
    A.nb = nb;
    track_init_kernel<<<1, 64, 0, s>>>(T, A.T64, A.counter, A.stat);
    for (int it = 0; it <= iters; ++it) {
        timer_begin("track_step", s);
        track_step_kernel<<<nb, kThreads, 0, s>>>(A, it);
        timer_end(s);
    }
    timer_begin("track_final", s);
    track_final_kernel<<<1, kThreads, 0, s>>>(A, iters);
    timer_end(s);
    return hipGetLastError();
}

hipError_t launch_fuse(int N, const float* T, float* Xc, float* Cc, const float* X, const float* C, hipStream_t s) {
    auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool vec = al16(Xc) && al16(Cc) && al16(X) && al16(C);
    const int quads = vec ? N / 4 : 0;
    const int tail = N - 4 * quads;
    if (quads > 0) {
        timer_begin("fuse", s);
        fuse_kernel<4><<<(quads + 255) / 256, 256, 0, s>>>(N, 0, T, Xc, Cc, X, C);
        timer_end(s);
    }
    if (tail > 0) fuse_kernel<1><<<(tail + 255) / 256, 256, 0, s>>>(N, 4 * quads, T, Xc, Cc, X, C);
    return hipGetLastError();
}

}  // namespace m3s
