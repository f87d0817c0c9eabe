// Device-side building blocks of the gfx950 matcher: the per-edge argument
// block, the ray-record layout of the workspace, the bilinear ray sampler and
// the per-query Levenberg-Marquardt projection (MASt3R-SLAM, Sec. 3.2, Eq. 2).
// Shared by the single-pair and the batched kernels so both produce the same
// bits for the same edge.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m3s {

// Everything one edge needs on the device.  Lives in kernel arguments for the
// single-pair launch and in the workspace edge table for the batched launch.
struct EdgeArgs {
    int32_t H, W, D, K, r, levels;
    int32_t tiles_x, tiles_y;      // query tiles of this edge (batched path)
    int32_t tile_begin;            // first global tile id of this edge (batched path)
    float lambda0, conf_min, max_theta, max_dist;
    const float* Xii;
    const float* Xji;
    const float* Dii;
    const float* Dji;
    const float* Qii;              // nullptr: no confidence gate
    const float* Qji;
    const float* p_init;           // nullptr: identity initialisation
    const float4* rays;            // workspace: ray image, 36 B per reference pixel (planes P0, P1, Z)
    float* p;
    int32_t* idx;
    uint8_t* valid;
    float* theta;                  // may be nullptr
    float* xhat;                   // may be nullptr
};

// Ray record of reference pixel m: the unit ray R = X/|X| (zero for a
// non-finite or zero point) and its central-difference gradients Gx, Gy along
// x and y (one-sided at the border), nine floats held in three planes of the
// ray image, one after the other: P0 = {R.x, R.y, R.z, Gx.x} and
// P1 = {Gx.y, Gx.z, Gy.x, Gy.y} (a float4 per pixel each), then Z = Gy.z (a
// float per pixel).  36 bytes per pixel, no padding; each plane is written and
// read in contiguous rows.
constexpr int kRecP4 = 2;            // float4 planes
constexpr uint32_t kRecBytes = 36;   // bytes per pixel over the three planes

// Byte offset of plane Z in a ray image of H x W pixels (plane P1 is at half of it).
__device__ __forceinline__ uint32_t ray_zoff(int H, int W) { return (uint32_t)H * (uint32_t)W * 32u; }

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }

// Hardware reciprocal and reciprocal square root (v_rcp_f32 / v_rsq_f32, about
// 1 ulp).  The matcher's tolerances are orders of magnitude looser.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ float3 load_point(const float* __restrict__ X, long m) {
    return f3(X[3 * m + 0], X[3 * m + 1], X[3 * m + 2]);
}

__device__ __forceinline__ bool finite3(float3 v) {
    return isfinite(v.x) && isfinite(v.y) && isfinite(v.z);
}

// Unit ray of a point, zero for a non-finite or zero point.
__device__ __forceinline__ float3 unit_ray(float3 x) {
    float n2 = x.x * x.x + x.y * x.y + x.z * x.z;
    if (!(finite3(x) && n2 > 0.0f && isfinite(n2))) return f3(0.f, 0.f, 0.f);
    float inv = rsq(n2);
    return f3(x.x * inv, x.y * inv, x.z * inv);
}

// What the LM step needs from one evaluation of the ray error: the cost and
// the Gauss-Newton blocks J^T J (without damping) and J^T e.
struct Sample {
    float c;                // ray error |e|^2 (inf for a degenerate sample)
    float a00, a01, a11;    // J^T J
    float g0, g1;           // J^T e
};

// Ray records are read with buffer loads: one resource descriptor (base,
// byte size) in scalar registers, a 32-bit byte offset per lane, immediate
// offsets within a record.  Reads past the size return 0.  The host keeps
// 36 * H * W below 2^32.
using RayBuf = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ RayBuf ray_buffer(const float4* rec, int H, int W) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(rec), (short)0,
                                             (int)((uint32_t)H * (uint32_t)W * kRecBytes), 0x00020000);
}

__device__ __forceinline__ float4 rec_load(RayBuf rb, uint32_t byte_off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rb, byte_off, 0, 0));
}

__device__ __forceinline__ float rec_load1(RayBuf rb, uint32_t byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, byte_off, 0, 0));
}

// Ray error of Eq. 2 from the four ray records around p (A = (x0, y0),
// B = (x0+1, y0), C = (x0, y0+1), D = (x0+1, y0+1): plane P in A..D, plane Z
// in z[0..3] in the same order) with bilinear weights a, b.
// FULL = false evaluates the cost only (the last trial of the LM needs nothing
// else).  A degenerate sample (interpolated ray zero or not finite) costs +inf;
// its Jacobian blocks are then not meaningful, and they are never used: a
// trial of infinite cost is never accepted, and a degenerate starting sample
// gives a non-finite step, which the LM rejects without moving.
// What the Jacobian part of a sample needs from its ray part: the bilinear
// weights, the unit interpolated ray psi, 1/|r| and the residual e.
struct RayPart {
    float w00, w10, w01, w11;
    float p0, p1, p2, inv;
    float e0, e1, e2;
};

#define M3S_BL(i, c) (r.w00 * A[i].c + r.w10 * B[i].c + r.w01 * C[i].c + r.w11 * D[i].c)

// Ray part of a sample: the cost |e|^2 (+inf when degenerate).
__device__ __forceinline__ float ray_cost_from(const float4* A, const float4* B, const float4* C, const float4* D,
                                               float a, float b, float3 t, RayPart& r) {
    r.w00 = (1.f - a) * (1.f - b), r.w10 = a * (1.f - b), r.w01 = (1.f - a) * b, r.w11 = a * b;
    float rx = M3S_BL(0, x), ry = M3S_BL(0, y), rz = M3S_BL(0, z);
    float n2 = rx * rx + ry * ry + rz * rz;
    const bool ok = n2 > 0.0f && n2 < INFINITY;  // false for 0, +inf and NaN
    r.inv = rsq(n2);
    r.p0 = rx * r.inv, r.p1 = ry * r.inv, r.p2 = rz * r.inv;
    r.e0 = r.p0 - t.x, r.e1 = r.p1 - t.y, r.e2 = r.p2 - t.z;
    return ok ? r.e0 * r.e0 + r.e1 * r.e1 + r.e2 * r.e2 : INFINITY;
}

// Jacobian part of a sample: J^T J and J^T e from the interpolated gradients.
__device__ __forceinline__ void ray_jacobian_from(const float4* A, const float4* B, const float4* C,
                                                  const float4* D, const float* z, const RayPart& r, Sample& s) {
    float gxx = M3S_BL(0, w), gxy = M3S_BL(1, x), gxz = M3S_BL(1, y);
    float gyx = M3S_BL(1, z), gyy = M3S_BL(1, w), gyz = r.w00 * z[0] + r.w10 * z[1] + r.w01 * z[2] + r.w11 * z[3];
    float pgx = r.p0 * gxx + r.p1 * gxy + r.p2 * gxz;
    float pgy = r.p0 * gyx + r.p1 * gyy + r.p2 * gyz;
    // J = (I - psi psi^T) [gx gy] / |r|  (Supp. A, Eq. norm_jac)
    float jx0 = (gxx - r.p0 * pgx) * r.inv, jx1 = (gxy - r.p1 * pgx) * r.inv, jx2 = (gxz - r.p2 * pgx) * r.inv;
    float jy0 = (gyx - r.p0 * pgy) * r.inv, jy1 = (gyy - r.p1 * pgy) * r.inv, jy2 = (gyz - r.p2 * pgy) * r.inv;
    s.a00 = jx0 * jx0 + jx1 * jx1 + jx2 * jx2;
    s.a01 = jx0 * jy0 + jx1 * jy1 + jx2 * jy2;
    s.a11 = jy0 * jy0 + jy1 * jy1 + jy2 * jy2;
    s.g0 = jx0 * r.e0 + jx1 * r.e1 + jx2 * r.e2;
    s.g1 = jy0 * r.e0 + jy1 * r.e1 + jy2 * r.e2;
}
#undef M3S_BL

template <bool FULL>
__device__ __forceinline__ void ray_error_from(const float4* A, const float4* B, const float4* C, const float4* D,
                                               const float* z, float a, float b, float3 t, Sample& s) {
    RayPart r;
    s.c = ray_cost_from(A, B, C, D, a, b, t, r);
    if constexpr (FULL) ray_jacobian_from(A, B, C, D, z, r, s);
}

// Ray records from the workspace in global memory.
struct GlobalRays {
    RayBuf rb;
    int W;
    uint32_t zoff;  // byte offset of plane Z (twice that of plane P1)
    __device__ __forceinline__ GlobalRays(const float4* rays, int H, int W_)
        : rb(ray_buffer(rays, H, W_)), W(W_), zoff(ray_zoff(H, W_)) {}
    __device__ __forceinline__ void fetch(int x0, int y0, float4* A, float4* B, float4* C, float4* D,
                                          float* z) const {
        const uint32_t m00 = (uint32_t)y0 * (uint32_t)W + (uint32_t)x0, m01 = m00 + (uint32_t)W;
        const uint32_t o00 = m00 * 16u, o01 = m01 * 16u, p1 = zoff >> 1;
        A[0] = rec_load(rb, o00);
        B[0] = rec_load(rb, o00 + 16);
        C[0] = rec_load(rb, o01);
        D[0] = rec_load(rb, o01 + 16);
        A[1] = rec_load(rb, p1 + o00);
        B[1] = rec_load(rb, p1 + o00 + 16);
        C[1] = rec_load(rb, p1 + o01);
        D[1] = rec_load(rb, p1 + o01 + 16);
        z[0] = rec_load1(rb, zoff + 4 * m00);
        z[1] = rec_load1(rb, zoff + 4 * m00 + 4);
        z[2] = rec_load1(rb, zoff + 4 * m01);
        z[3] = rec_load1(rb, zoff + 4 * m01 + 4);
    }
};

// Ray records of a window [rx0, rx0 + rw) x [ry0, ry0 + rh) staged in LDS:
// planes P0 and P1 of window pixel k at lds[2k] and lds[2k + 1], plane Z at
// ldz[k] (ldz = lds + 2 rw rh); cells outside the window are read from global
// memory.  Same values either way.
struct WindowRays {
    const float4* lds;
    const float* ldz;
    int rx0, ry0, rw, rh;
    GlobalRays g;
    __device__ __forceinline__ WindowRays(const float4* l, int x, int y, int w, int h, const GlobalRays& g_)
        : lds(l), ldz(reinterpret_cast<const float*>(l + kRecP4 * w * h)), rx0(x), ry0(y), rw(w), rh(h), g(g_) {}
    __device__ __forceinline__ void fetch(int x0, int y0, float4* A, float4* B, float4* C, float4* D,
                                          float* z) const {
        const int lx = x0 - rx0, ly = y0 - ry0;
        // 0 <= lx <= rw - 2 and 0 <= ly <= rh - 2 (the whole cell in the window).
        if ((uint32_t)lx < (uint32_t)(rw - 1) && (uint32_t)ly < (uint32_t)(rh - 1)) {
            const uint32_t k = (uint32_t)(ly * rw + lx);
            const float4* a = lds + kRecP4 * k;
            const float4* c = a + kRecP4 * rw;
#pragma unroll
            for (int j = 0; j < kRecP4; ++j) {
                A[j] = a[j];
                B[j] = a[kRecP4 + j];
                C[j] = c[j];
                D[j] = c[kRecP4 + j];
            }
            const float* zz = ldz + k;
            z[0] = zz[0];
            z[1] = zz[1];
            z[2] = zz[rw];
            z[3] = zz[rw + 1];
        } else {
            g.fetch(x0, y0, A, B, C, D, z);
        }
    }
};

// Ray error of Eq. 2 at pixel (px, py) (inside the domain) for target ray t.
// The cell origin is min(floor(p), size - 2), formed in fp32 (exact for
// integers), so p = size - 1 lies on the last cell's far edge.
template <bool FULL = true, class Src>
__device__ __forceinline__ void sample_ray_error(const Src& src, float xcell, float ycell, float px, float py,
                                                 float3 t, Sample& s) {
    const float fx0 = fminf(floorf(px), xcell), fy0 = fminf(floorf(py), ycell);
    const float a = px - fx0, b = py - fy0;
    float4 A[kRecP4], B[kRecP4], C[kRecP4], D[kRecP4];
    float z[4];
    src.fetch((int)fx0, (int)fy0, A, B, C, D, z);
    ray_error_from<FULL>(A, B, C, D, z, a, b, t, s);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }

// Levenberg-Marquardt state of one query: current pixel, damping and the
// sample at the current pixel.
struct LMState {
    float px, py, lambda;
    Sample cur;
};

template <class Src>
__device__ __forceinline__ void lm_start(const Src& src, int H, int W, float lambda0, float3 t, LMState& st) {
    sample_ray_error(src, (float)(W - 2), (float)(H - 2), st.px, st.py, t, st.cur);
    st.lambda = lambda0;
}

// Damped 2x2 step of Eq. 2's normal equations at the current state; false
// when it is not finite.  A coordinate on its bound whose step points out of
// the image is held, and the other coordinate takes its own 1-D damped step.
// Returns the clamped trial pixel.
__device__ __forceinline__ bool lm_step(const Sample& cur, float lambda, float px, float py, float xmax, float ymax,
                                        float& qx, float& qy) {
    float a00 = cur.a00 + lambda, a01 = cur.a01, a11 = cur.a11 + lambda;
    float g0 = cur.g0, g1 = cur.g1;
    float idet = rcp(a00 * a11 - a01 * a01);
    float dx = -(a11 * g0 - a01 * g1) * idet;
    float dy = -(a00 * g1 - a01 * g0) * idet;
    if (!isfinite(dx) || !isfinite(dy)) return false;
    bool hold_x = (px <= 0.f && dx < 0.f) || (px >= xmax && dx > 0.f);
    bool hold_y = (py <= 0.f && dy < 0.f) || (py >= ymax && dy > 0.f);
    if (__builtin_expect(hold_x | hold_y, 0)) {
        float fx = -g0 * rcp(a00), fy = -g1 * rcp(a11);
        dx = hold_x ? 0.f : fx;
        dy = hold_y ? 0.f : fy;
    }
    qx = clampf(px + dx, 0.f, xmax);
    qy = clampf(py + dy, 0.f, ymax);
    return true;
}

// `iters` LM iterations on Eq. 2: damped 2x2 step, bound hold, clamp,
// acceptance on strictly lower cost.  With `final` set these are the last
// iterations of the query, and the last trial evaluates its cost only.
// UNROLL: unroll factor of the iteration loop (a launch-shape choice of the
// autotuner; the arithmetic, and so every output bit, is the same).
template <int UNROLL = 1, class Src>
__device__ __forceinline__ void lm_iterate(const Src& src, int H, int W, float3 t, int iters, LMState& st,
                                           bool final = true) {
    const float xmax = (float)(W - 1), ymax = (float)(H - 1);
    const float xcell = (float)(W - 2), ycell = (float)(H - 2);
    float px = st.px, py = st.py, lambda = st.lambda;
    Sample cur = st.cur, nxt;
    const int full = final ? iters - 1 : iters;
#pragma unroll UNROLL
    for (int it = 0; it < full; ++it) {
        float qx, qy;
        if (!lm_step(cur, lambda, px, py, xmax, ymax, qx, qy)) { lambda *= 10.f; continue; }
        // The trial's cost first; its Jacobian blocks only where it is accepted
        // (on strictly lower cost).  After the first few iterations most lanes
        // reject, and a wave whose lanes all reject skips that part.
        const float fx0 = fminf(floorf(qx), xcell), fy0 = fminf(floorf(qy), ycell);
        float4 A[kRecP4], B[kRecP4], C[kRecP4], D[kRecP4];
        float z[4];
        src.fetch((int)fx0, (int)fy0, A, B, C, D, z);
        RayPart r;
        const float c = ray_cost_from(A, B, C, D, qx - fx0, qy - fy0, t, r);
        const bool acc = c < cur.c;
        if (acc) {
            ray_jacobian_from(A, B, C, D, z, r, cur);
            cur.c = c;
            px = qx;
            py = qy;
        }
        lambda = acc ? lambda * 0.1f : lambda * 10.f;
    }
    if (final && iters > 0) {
        float qx, qy;
        if (lm_step(cur, lambda, px, py, xmax, ymax, qx, qy)) {
            sample_ray_error<false>(src, xcell, ycell, qx, qy, t, nxt);
            const bool acc = nxt.c < cur.c;
            px = acc ? qx : px;
            py = acc ? qy : py;
            cur.c = acc ? nxt.c : cur.c;
        }
    }
    st.px = px; st.py = py; st.lambda = lambda; st.cur = cur;
}

// K Levenberg-Marquardt iterations from (px, py) reading global memory; returns the final cost.
__device__ __forceinline__ float lm_project(const float4* __restrict__ rays, int H, int W, int K, float lambda0,
                                            float3 t, float& px, float& py) {
    const GlobalRays g(rays, H, W);
    LMState st;
    st.px = px; st.py = py;
    lm_start(g, H, W, lambda0, t, st);
    lm_iterate(g, H, W, t, K, st);
    px = st.px; py = st.py;
    return st.cur.c;
}

}  // namespace m3s
