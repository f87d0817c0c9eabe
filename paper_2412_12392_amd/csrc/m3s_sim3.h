// Device helpers shared by the pose solves (MASt3R-SLAM, Sec. 3.3 and 3.5):
// Sim(3) algebra in fp64 and the per-match accumulation of the ray and
// distance normal equations in fp32.
//
// Pose layout: row-major 3x4 [sR | t].  Tangent order tau = (v, omega, sigma),
// matching the point Jacobian [I, -[x]_x, x] of Supp. A; updates are left plus,
// T <- Exp(tau) o T (Eq. 1).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace m3s {

// Number of accumulated values per match set: the upper triangle of the 7x7
// J^T W J (28, rows of 7, 6, ..., 1), J^T W r (7), robust cost, match count.
constexpr int kPoseVals = 28 + 7 + 2;

__device__ __forceinline__ constexpr int upper_index(int a, int b) { return a * 7 - a * (a - 1) / 2 + (b - a); }

// Huber weight and cost of a whitened norm a with the given width.
__device__ __forceinline__ float huber_weight(float a, float width) { return a <= width ? 1.f : width / a; }
__device__ __forceinline__ float huber_cost(float a, float width) {
    return a <= width ? 0.5f * a * a : width * (a - 0.5f * width);
}

// Weights of the two residual blocks: 1 / sigma^2 and 1 / sigma (0 drops the
// residual), and the Huber width.
struct RobustWeights {
    float w_ray, w_dist, is_ray, is_dist, huber;
};

inline RobustWeights robust_weights(float sigma_ray, float sigma_dist, float huber) {
    RobustWeights w;
    w.w_ray = isinf(sigma_ray) ? 0.f : 1.f / (sigma_ray * sigma_ray);
    w.w_dist = isinf(sigma_dist) ? 0.f : 1.f / (sigma_dist * sigma_dist);
    w.is_ray = isinf(sigma_ray) ? 0.f : 1.f / sigma_ray;
    w.is_dist = isinf(sigma_dist) ? 0.f : 1.f / sigma_dist;
    w.huber = huber;
    return w;
}

// Confidence gate of a match (Sec. 3.3): q = sqrt(Qa Qb) > q_min, decided
// exactly as in fp64 (the product of two fp32 values is exact there).  The
// fp32 root is within 2 ulp of the exact one, so outside a relative band of
// 1e-5 around q_min its comparison gives the fp64 answer; inside the band the
// fp64 root decides.  Writes the fp32 confidence to q.
__device__ __forceinline__ bool confidence_gate(float Qa, float Qb, double q_min, float q_minf, float& q) {
    q = sqrtf(Qa * Qb);
    if (fabsf(q - q_minf) > 1e-5f * q_minf) return q > q_minf;
    return sqrt((double)Qa * (double)Qb) > q_min;
}

// One match: x = T X (X the point that moves with the pose), Y the measured
// point, q its confidence.  Ray residual e = psi(x) - psi(Y) and distance
// residual rd = |x| - |Y| (Sec. 3.3); their Jacobians w.r.t. a left
// perturbation of T (Supp. A) are J_ray = [P/d, -[x]_x/d, 0] and
// J_dist = [u^T, 0, d] with d = |x|, u = x/d and the projector P = I - u u^T;
// weights wr = q/sigma_ray^2 and wd = q/sigma_dist^2, each times the Huber
// weight of its whitened block norm |r| sqrt(q)/sigma.  Since P^T P = P,
// P [x]_x = [x]_x and [x]_x^T [x]_x = d^2 P, the weighted normal equations
// have the closed form (ar = wr/d^2)
//   H_vv = ar I + (wd - ar) u u^T   H_vw = -ar [x]_x   H_vs = wd d u
//   H_ww = wr P                     H_ws = 0           H_ss = wd d^2
//   g_v  = wr P e / d + wd rd u     g_w = wr u x e     g_s  = wd rd d
// which is what is added to acc (upper triangle of H by rows, then g, the
// robust cost and the count).  Returns false, adding nothing, for a point at
// the origin or non-finite.
__device__ __forceinline__ bool accumulate_match(const float* T, float X0, float X1, float X2, float Y0, float Y1,
                                                 float Y2, float q, const RobustWeights& rw, float* acc) {
    const float x0 = T[0] * X0 + T[1] * X1 + T[2] * X2 + T[3];
    const float x1 = T[4] * X0 + T[5] * X1 + T[6] * X2 + T[7];
    const float x2 = T[8] * X0 + T[9] * X1 + T[10] * X2 + T[11];
    const float d = sqrtf(x0 * x0 + x1 * x1 + x2 * x2);
    const float dy = sqrtf(Y0 * Y0 + Y1 * Y1 + Y2 * Y2);
    if (!(d > 0.f) || !(dy > 0.f) || !isfinite(d) || !isfinite(dy)) return false;
    const float id = __builtin_amdgcn_rcpf(d), idy = __builtin_amdgcn_rcpf(dy);
    const float u0 = x0 * id, u1 = x1 * id, u2 = x2 * id;
    const float e0 = u0 - Y0 * idy, e1 = u1 - Y1 * idy, e2 = u2 - Y2 * idy, rd = d - dy;
    const float sq = sqrtf(q);
    const float a_ray = sqrtf(e0 * e0 + e1 * e1 + e2 * e2) * sq * rw.is_ray;
    const float a_dist = fabsf(rd) * sq * rw.is_dist;
    const float hr = a_ray <= rw.huber ? 1.f : rw.huber * __builtin_amdgcn_rcpf(a_ray);
    const float hd = a_dist <= rw.huber ? 1.f : rw.huber * __builtin_amdgcn_rcpf(a_dist);
    const float wr = q * rw.w_ray * hr;
    const float wd = q * rw.w_dist * hd;
    const float ar = wr * id * id;
    const float cv = wd - ar;
    const float wdd = wd * d;
    // H_vv, H_vw, H_vs (rows 0..2)
    acc[upper_index(0, 0)] += ar + cv * u0 * u0;
    acc[upper_index(0, 1)] += cv * u0 * u1;
    acc[upper_index(0, 2)] += cv * u0 * u2;
    acc[upper_index(0, 4)] += ar * x2;
    acc[upper_index(0, 5)] -= ar * x1;
    acc[upper_index(0, 6)] += wdd * u0;
    acc[upper_index(1, 1)] += ar + cv * u1 * u1;
    acc[upper_index(1, 2)] += cv * u1 * u2;
    acc[upper_index(1, 3)] -= ar * x2;
    acc[upper_index(1, 5)] += ar * x0;
    acc[upper_index(1, 6)] += wdd * u1;
    acc[upper_index(2, 2)] += ar + cv * u2 * u2;
    acc[upper_index(2, 3)] += ar * x1;
    acc[upper_index(2, 4)] -= ar * x0;
    acc[upper_index(2, 6)] += wdd * u2;
    // H_ww (rows 3..5), H_ss
    acc[upper_index(3, 3)] += wr - wr * u0 * u0;
    acc[upper_index(3, 4)] -= wr * u0 * u1;
    acc[upper_index(3, 5)] -= wr * u0 * u2;
    acc[upper_index(4, 4)] += wr - wr * u1 * u1;
    acc[upper_index(4, 5)] -= wr * u1 * u2;
    acc[upper_index(5, 5)] += wr - wr * u2 * u2;
    acc[upper_index(6, 6)] += wdd * d;
    // g
    const float ue = u0 * e0 + u1 * e1 + u2 * e2;
    const float wri = wr * id, wdr = wd * rd;
    acc[28] += wri * (e0 - u0 * ue) + wdr * u0;
    acc[29] += wri * (e1 - u1 * ue) + wdr * u1;
    acc[30] += wri * (e2 - u2 * ue) + wdr * u2;
    acc[31] += wr * (u1 * e2 - u2 * e1);
    acc[32] += wr * (u2 * e0 - u0 * e2);
    acc[33] += wr * (u0 * e1 - u1 * e0);
    acc[34] += wdr * d;
    acc[35] += huber_cost(a_ray, rw.huber) + huber_cost(a_dist, rw.huber);
    acc[36] += 1.f;
    return true;
}

// Fixed-order fp64 sum of nparts fp32 partials of kPoseVals values each
// (stride `stride` floats) by a workgroup of NT threads: G = NT / kPoseVals
// groups of kPoseVals threads, thread (g, v) adding value v of the partials
// g, g + G, g + 2G, ... in that order (a group's reads of one partial are
// contiguous, and every group's reads are in flight together); then thread v
// adds the G group sums in group order.  `part` is LDS of G * kPoseVals
// doubles; the sums land in out[0 .. kPoseVals) (LDS), visible to the whole
// workgroup on return.
template <int NT>
__device__ void sum_partials(const float* __restrict__ parts, int nparts, int stride, double* part, double* out) {
    constexpr int G = NT / kPoseVals;
    static_assert(G >= 1, "one thread per value at least");
    const int t = threadIdx.x, g = t / kPoseVals, v = t - g * kPoseVals;
    if (g < G) {
        double acc = 0.0;
#pragma unroll 8
        for (int b = g; b < nparts; b += G) acc += (double)parts[(size_t)b * stride + v];
        part[g * kPoseVals + v] = acc;
    }
    __syncthreads();
    if (t < kPoseVals) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < G; ++k) s += part[k * kPoseVals + t];
        out[t] = s;
    }
    __syncthreads();
}

// Sum over the 64 lanes of a wave (every lane active), in every lane: DPP quad
// swaps, half-row and row mirrors give each row's sum in its lanes, then the
// four row sums are added in a fixed order.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Scale of a similarity [sR | t]: the cube root of det(sR).
__device__ inline double sim3_scale(const double* T) {
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    return cbrt(det);
}

// out = T^-1 = [R^T / s | -R^T t / s].
__device__ inline void sim3_inverse(const double* T, double* out) {
    const double s = sim3_scale(T), s2 = s * s;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[4 * i + j] = T[4 * j + i] / s2;
    for (int i = 0; i < 3; ++i)
        out[4 * i + 3] = -(out[4 * i] * T[3] + out[4 * i + 1] * T[7] + out[4 * i + 2] * T[11]);
}

// out = A B (out must not alias A or B).
__device__ inline void sim3_mul(const double* A, const double* B, double* out) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j)
            out[4 * i + j] = A[4 * i] * B[j] + A[4 * i + 1] * B[4 + j] + A[4 * i + 2] * B[8 + j] +
                             (j == 3 ? A[4 * i + 3] : 0.0);
}

// Ad(T) on (v, omega, sigma): [[sR, [t]_x R, -t], [0, R, 0], [0, 0, 1]], row-major 7x7.
__device__ inline void sim3_adjoint(const double* T, double* A) {
    const double s = sim3_scale(T);
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = T[4 * i + j] / s;
    const double t[3] = {T[3], T[7], T[11]};
    const double S[3][3] = {{0.0, -t[2], t[1]}, {t[2], 0.0, -t[0]}, {-t[1], t[0], 0.0}};
    for (int k = 0; k < 49; ++k) A[k] = 0.0;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            A[7 * i + j] = s * R[i][j];
            A[7 * i + 3 + j] = S[i][0] * R[0][j] + S[i][1] * R[1][j] + S[i][2] * R[2][j];
            A[7 * (3 + i) + 3 + j] = R[i][j];
        }
        A[7 * i + 6] = -t[i];
    }
    A[48] = 1.0;
}

// Exp of sim(3): tau = (v, omega, sigma) -> [e^sigma R | V v], R by Rodrigues
// and V = a0 I + a1 [omega]_x + a2 [omega]_x^2 with a0 = int e^{sigma s},
// a1 = int e^{sigma s} sin(theta s) / theta and
// a2 = int e^{sigma s} (1 - cos(theta s)) / theta^2 over s in [0, 1]; their
// series near theta = 0 and sigma = 0.
__device__ inline void sim3_exp(const double* tau, double* E) {
    const double sg = tau[6];
    const double w0 = tau[3], w1 = tau[4], w2 = tau[5];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    const double S[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double S2[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S2[i][j] = S[i][0] * S[0][j] + S[i][1] * S[1][j] + S[i][2] * S[2][j];
    double sn, cs;
    sincos(th, &sn, &cs);
    const bool small = th < 1e-4;
    const double ka = small ? 1.0 - th2 / 6.0 : sn / th;
    const double kb = small ? 0.5 - th2 / 24.0 : (1.0 - cs) / th2;
    const double es = exp(sg);
    const double a0 = sg == 0.0 ? 1.0 : expm1(sg) / sg;
    double a1, a2;
    if (small) {
        const double s2 = sg * sg;
        if (fabs(sg) < 1e-3) {
            a1 = 0.5 + sg / 3.0 + s2 / 8.0 + s2 * sg / 30.0;
            a2 = 1.0 / 6.0 + sg / 8.0 + s2 / 20.0 + s2 * sg / 72.0;
        } else {
            a1 = (es * (sg - 1.0) + 1.0) / s2;
            a2 = (es * (s2 - 2.0 * sg + 2.0) - 2.0) / (2.0 * s2 * sg);
        }
    } else {
        const double den = sg * sg + th2;
        const double is = (es * (sg * sn - th * cs) + th) / den;
        const double ic = (es * (sg * cs + th * sn) - sg) / den;
        a1 = is / th;
        a2 = (a0 - ic) / th2;
    }
    for (int i = 0; i < 3; ++i) {
        double tv = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            E[4 * i + j] = es * (I + ka * S[i][j] + kb * S2[i][j]);
            tv += (I * a0 + a1 * S[i][j] + a2 * S2[i][j]) * tau[j];
        }
        E[4 * i + 3] = tv;
    }
}

}  // namespace m3s
