// gfx950 kernels of the projective pointmap matcher (MASt3R-SLAM, Sec. 3.2).
//
//   prep      ray image R = X^i_i / |X^i_i| and its central-difference
//             gradient images, 36 B per reference pixel in three planes
//             (Sec. 3.1: each pointmap defines its own central camera through
//             its rays; Fig. 2: the reference pointmap is normalised first).
//   fwd       one lane per query pixel: LM on the ray error (Eq. 2), residual
//             angle (Eq. 3), bilinear xhat, window refine by descriptor dot
//             product (feature refinement paragraph), gates (Sec. 3.2, 3.3).
//   bwd       implicit adjoint at p*, scattered into dL/dX^i_i through an LDS
//             window of 64-bit fixed point.
//   batched   persistent work-queue version of prep + fwd over an edge table.
//
// Every launch is checked on the host against the shapes its grid assumes;
// kernels bound-check every pixel they touch against H and W.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <climits>
#include <type_traits>

#include "m3s_device.h"
#include "m3s_internal.h"

namespace m3s {

// ---------------------------------------------------------------- prep

// Streaming 16-byte store (non-temporal hint: the line is not kept dirty in
// this XCD's L2 for a later write-back).
typedef float f4v_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt(float4* p, float4 v) {
    __builtin_nontemporal_store(__builtin_bit_cast(f4v_t, v), reinterpret_cast<f4v_t*>(p));
}
__device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

// One prep tile of kPrepTX x kPrepTY pixels per workgroup of 256 lanes.  The
// tile and a one-pixel halo of X (edge-replicated, which gives the one-sided
// differences at the image border) are read with coalesced loads, each
// pixel's unit ray is computed once in LDS, and each lane writes its pixels'
// records to the three planes (a wave writes contiguous rows of each).  Same
// arithmetic per pixel as reading the five points directly: r, rx-, rx+, ry-,
// ry+ and (r+ - r-) / (x+ - x-).
struct PrepLds {
    float ray[(kPrepTY + 2) * (kPrepTX + 2) * 3];
};

__device__ __forceinline__ void prep_tile(const float* __restrict__ X, float4* __restrict__ rec, int H, int W,
                                          int tile, PrepLds& S) {
    constexpr int HW_ = kPrepTX + 2, HROW = HW_ * 3;
    const int tid = threadIdx.x;
    const int tiles_x = (W + kPrepTX - 1) / kPrepTX;
    const int x0 = (tile % tiles_x) * kPrepTX, y0 = (tile / tiles_x) * kPrepTY;
    for (int i = tid; i < (kPrepTY + 2) * HROW; i += 256) {
        const int j = i / HROW, rem = i - j * HROW, c = rem / 3, k = rem - 3 * c;
        const int y = min(max(y0 - 1 + j, 0), H - 1), x = min(max(x0 - 1 + c, 0), W - 1);
        S.ray[i] = X[((long)y * W + x) * 3 + k];
    }
    __syncthreads();
    for (int i = tid; i < (kPrepTY + 2) * HW_; i += 256) {
        const float3 r = unit_ray(f3(S.ray[3 * i], S.ray[3 * i + 1], S.ray[3 * i + 2]));
        S.ray[3 * i] = r.x; S.ray[3 * i + 1] = r.y; S.ray[3 * i + 2] = r.z;
    }
    __syncthreads();
    for (int pix = tid; pix < kPrepTX * kPrepTY; pix += 256) {
        const int lx = pix % kPrepTX, ly = pix / kPrepTX;
        const int x = x0 + lx, y = y0 + ly;
        const int xm = max(x - 1, 0), xp = min(x + 1, W - 1);
        const int ym = max(y - 1, 0), yp = min(y + 1, H - 1);
        // Halo column of pixel x' is x' - x0 + 1 (clamped like the load above).
        auto at = [&](int yy, int xx) {
            const float* q = S.ray + 3 * ((yy - y0 + 1) * HW_ + (xx - x0 + 1));
            return f3(q[0], q[1], q[2]);
        };
        if (x < W && y < H) {
            const float3 r = at(y, x), rxm = at(y, xm), rxp = at(y, xp), rym = at(ym, x), ryp = at(yp, x);
            float sx = 1.0f / (float)(xp - xm), sy = 1.0f / (float)(yp - ym);
            float3 gx = f3((rxp.x - rxm.x) * sx, (rxp.y - rxm.y) * sx, (rxp.z - rxm.z) * sx);
            float3 gy = f3((ryp.x - rym.x) * sy, (ryp.y - rym.y) * sy, (ryp.z - rym.z) * sy);
            const long m = (long)y * W + x, hw = (long)H * W;
            store_nt(rec + m, make_float4(r.x, r.y, r.z, gx.x));
            store_nt(rec + hw + m, make_float4(gx.y, gx.z, gy.x, gy.y));
            store_nt(reinterpret_cast<float*>(rec + 2 * hw) + m, gy.z);
        }
    }
}

__global__ void __launch_bounds__(256) prep_kernel(const float* __restrict__ X, float4* __restrict__ rec, int H, int W) {
    __shared__ PrepLds S;
    prep_tile(X, rec, H, W, blockIdx.x, S);
}

// Tile of workgroup b in a 1-D launch over `tiles` tiles.  Workgroups are
// dispatched to the 8 XCDs round-robin, so with remap on, XCD j (b % 8 == j)
// takes the j-th contiguous band of tiles and neighbouring tiles share that
// XCD's L2; returns -1 for the padding workgroups of the last band.
constexpr int kXcds = 8;
__device__ __forceinline__ int tile_of_block(int b, int tiles, bool remap) {
    if (!remap) return b < tiles ? b : -1;
    const int per = (tiles + kXcds - 1) / kXcds;
    const int t = (b % kXcds) * per + b / kXcds;
    return t < tiles ? t : -1;
}

// Fallback-path counters (indices kPath*, read by read_path_counters): one
// vector atomic per tile (per query for kPathRefineQuery) that leaves its
// fast path, so tests can show that every branch ran.
__device__ unsigned long long g_path_counts[kNumPathCounters];

__device__ __forceinline__ void count_path(int k) { atomicAdd(&g_path_counts[k], 1ull); }

// ---------------------------------------------------------------- forward

// Descriptor dot product of the query (in registers for a compile-time D)
// with reference pixel m; the products are accumulated in index order.
template <int DT>
struct QueryDesc {
    float q[DT];
    __device__ __forceinline__ void load(const float* __restrict__ Dj, long n, int) {
        const float4* s = reinterpret_cast<const float4*>(Dj + (long)DT * n);
#pragma unroll
        for (int k = 0; k < DT / 4; ++k) {
            float4 v = s[k];
            q[4 * k] = v.x; q[4 * k + 1] = v.y; q[4 * k + 2] = v.z; q[4 * k + 3] = v.w;
        }
    }
    __device__ __forceinline__ float dot(const float* __restrict__ Di, long m, int) const {
        const float4* s = reinterpret_cast<const float4*>(Di + (long)DT * m);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < DT / 4; ++k) {
            float4 v = s[k];
            acc = fmaf(q[4 * k], v.x, acc);
            acc = fmaf(q[4 * k + 1], v.y, acc);
            acc = fmaf(q[4 * k + 2], v.z, acc);
            acc = fmaf(q[4 * k + 3], v.w, acc);
        }
        return acc;
    }
};

// Any D (or unaligned descriptors): both operands read from memory.
template <>
struct QueryDesc<0> {
    const float* q;
    __device__ __forceinline__ void load(const float* __restrict__ Dj, long n, int D) { q = Dj + (long)D * n; }
    __device__ __forceinline__ float dot(const float* __restrict__ Di, long m, int D) const {
        const float* d = Di + (long)D * m;
        float acc = 0.f;
        for (int k = 0; k < D; ++k) acc = fmaf(q[k], d[k], acc);
        return acc;
    }
};

// Per-query state between the phases of the forward.
struct QState {
    float px, py;     // p* (clamped to the image)
    float th;         // residual angle
    float3 xq;        // query point x_n
    bool good;        // finite, non-zero query point and initial pixel
};

// Phase 1a: query setup.  Reads x_n and the initial pixel; a bad query gets
// its final outputs here and returns false.
__device__ __forceinline__ bool lm_setup(const EdgeArgs& A, int x, int y, QState& q, float3& t, LMState& st) {
    const int H = A.H, W = A.W;
    const long n = (long)y * W + x;
    float3 xq = load_point(A.Xji, n);
    float px0, py0;
    bool bad = false;
    if (A.p_init) {
        px0 = A.p_init[2 * n];
        py0 = A.p_init[2 * n + 1];
        if (!isfinite(px0) || !isfinite(py0)) { bad = true; px0 = py0 = 0.f; }
    } else {
        px0 = (float)x;
        py0 = (float)y;
    }
    float px = clampf(px0, 0.f, (float)(W - 1)), py = clampf(py0, 0.f, (float)(H - 1));
    float n2 = xq.x * xq.x + xq.y * xq.y + xq.z * xq.z;
    if (!finite3(xq) || !(n2 > 0.f) || !isfinite(n2)) bad = true;
    q.xq = xq;
    q.good = !bad;
    q.px = px; q.py = py; q.th = INFINITY;
    if (bad) {
        reinterpret_cast<float2*>(A.p)[n] = make_float2(px, py);
        A.idx[n] = -1;
        A.valid[n] = 0;
        if (A.theta) A.theta[n] = INFINITY;
        if (A.xhat) { A.xhat[3 * n] = NAN; A.xhat[3 * n + 1] = NAN; A.xhat[3 * n + 2] = NAN; }
        return false;
    }
    float inv = rsq(n2);
    t = f3(xq.x * inv, xq.y * inv, xq.z * inv);
    st.px = px;
    st.py = py;
    return true;
}

// Phase 1c: outputs of the LM: p*, residual angle (Eq. 3 solved for theta), xhat.
__device__ __forceinline__ void lm_finish(const EdgeArgs& A, int x, int y, const LMState& st, QState& q) {
    const int H = A.H, W = A.W;
    const long n = (long)y * W + x;
    const float px = st.px, py = st.py;
    reinterpret_cast<float2*>(A.p)[n] = make_float2(px, py);
    float th = 2.0f * asinf(fminf(1.0f, sqrtf(st.cur.c) * 0.5f));
    if (A.theta) A.theta[n] = th;
    if (A.xhat) {
        int x0 = min((int)floorf(px), W - 2), y0 = min((int)floorf(py), H - 2);
        float a = px - (float)x0, b = py - (float)y0;
        long m00 = (long)y0 * W + x0;
        float3 X00 = load_point(A.Xii, m00), X10 = load_point(A.Xii, m00 + 1);
        float3 X01 = load_point(A.Xii, m00 + W), X11 = load_point(A.Xii, m00 + W + 1);
        float w00 = (1.f - a) * (1.f - b), w10 = a * (1.f - b), w01 = (1.f - a) * b, w11 = a * b;
        A.xhat[3 * n + 0] = w00 * X00.x + w10 * X10.x + w01 * X01.x + w11 * X11.x;
        A.xhat[3 * n + 1] = w00 * X00.y + w10 * X10.y + w01 * X01.y + w11 * X11.y;
        A.xhat[3 * n + 2] = w00 * X00.z + w10 * X10.z + w01 * X01.z + w11 * X11.z;
    }
    q.px = px; q.py = py; q.th = th;
}

// Phase 1 through global memory: LM on Eq. 2, residual angle and xhat.
__device__ __forceinline__ void lm_phase(const EdgeArgs& A, int x, int y, QState& q) {
    float3 t;
    LMState st;
    if (!lm_setup(A, x, y, q, t, st)) return;
    const GlobalRays g(A.rays, A.H, A.W);
    lm_start(g, A.H, A.W, A.lambda0, t, st);
    lm_iterate(g, A.H, A.W, t, A.K, st);
    lm_finish(A, x, y, st, q);
}

// Refine window centre: p* rounded half up.
__device__ __forceinline__ int round_half_up(float v) { return (int)floorf(v + 0.5f); }

// One level of the window refine through global memory: the first maximum
// of the raw dot product over the (2r+1)^2 grid of spacing sp around
// (mx0, my0), in row-major order, skipping candidates outside the image; -1
// when none is inside.
template <int DT>
__device__ __forceinline__ long refine_global_level(const EdgeArgs& A, const QueryDesc<DT>& qd, int mx0, int my0,
                                                    int sp) {
    const int H = A.H, W = A.W, r = A.r;
    float best = -INFINITY;
    long lb = -1;
    for (int dy = -r; dy <= r; ++dy) {
        int my = my0 + sp * dy;
        if (my < 0 || my >= H) continue;
        for (int dx = -r; dx <= r; ++dx) {
            int mx = mx0 + sp * dx;
            if (mx < 0 || mx >= W) continue;
            long m = (long)my * W + mx;
            float s = qd.dot(A.Dii, m, A.D);
            if (s > best) { best = s; lb = m; }
        }
    }
    return lb;
}

// Phase 2 (global memory): first maximum of the raw dot product over the
// window; with L > 1 levels, coarse to fine: level l scans the grid of
// spacing 2^l around the previous level's best.
template <int DT>
__device__ __forceinline__ long refine_global(const EdgeArgs& A, long n, const QState& q) {
    const int W = A.W;
    int mx0 = round_half_up(q.px), my0 = round_half_up(q.py);
    QueryDesc<DT> qd;
    qd.load(A.Dji, n, A.D);
    long bi = -1;
    for (int lev = A.levels - 1; lev >= 0; --lev) {
        const long lb = refine_global_level<DT>(A, qd, mx0, my0, 1 << lev);
        if (lb < 0) break;
        bi = lb;
        mx0 = (int)(lb % W);
        my0 = (int)(lb / W);
    }
    return bi;
}

// Phase 2 (LDS): the same scan over a staged region of D^i_i held as six
// float4 planes (plane k holds descriptor floats 4k..4k+3 of every region
// pixel at a stride of 16 bytes, so neighbouring lanes read neighbouring
// 16-byte words).  Same products in the same order as refine_global.
template <int REGION>
__device__ __forceinline__ long refine_lds(const EdgeArgs& A, long n, const QState& q, const float4* __restrict__ sdesc,
                                           int rx0, int ry0, int rw) {
    const int H = A.H, W = A.W, r = A.r;
    int mx0 = round_half_up(q.px), my0 = round_half_up(q.py);
    QueryDesc<24> qd;
    qd.load(A.Dji, n, 24);
    float best = -INFINITY;
    long bi = -1;
    for (int dy = -r; dy <= r; ++dy) {
        int my = my0 + dy;
        if (my < 0 || my >= H) continue;
        const int row = (my - ry0) * rw - rx0;
        for (int dx = -r; dx <= r; ++dx) {
            int mx = mx0 + dx;
            if (mx < 0 || mx >= W) continue;
            const float4* d = sdesc + row + mx;
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                float4 v = d[k * REGION];
                acc = fmaf(qd.q[4 * k], v.x, acc);
                acc = fmaf(qd.q[4 * k + 1], v.y, acc);
                acc = fmaf(qd.q[4 * k + 2], v.z, acc);
                acc = fmaf(qd.q[4 * k + 3], v.w, acc);
            }
            if (acc > best) { best = acc; bi = (long)my * W + mx; }
        }
    }
    return bi;
}

// Phase 3: gates (residual angle, match confidence of Sec. 3.3, 3D distance
// of Sec. 3.2) and the refined index.
__device__ __forceinline__ void finish(const EdgeArgs& A, long n, const QState& q, long bi) {
    bool ok = bi >= 0 && q.th <= A.max_theta;
    if (ok && A.Qii) ok = sqrtf(A.Qii[bi] * A.Qji[n]) >= A.conf_min;
    if (ok && A.max_dist < INFINITY) {
        float3 xr = load_point(A.Xii, bi);
        float d0 = xr.x - q.xq.x, d1 = xr.y - q.xq.y, d2 = xr.z - q.xq.z;
        ok = sqrtf(d0 * d0 + d1 * d1 + d2 * d2) <= A.max_dist;
    }
    A.idx[n] = (int32_t)bi;
    A.valid[n] = ok ? 1 : 0;
}

// One query end to end through global memory.
template <int DT>
__device__ __forceinline__ void match_query(const EdgeArgs& A, int x, int y) {
    QState q;
    lm_phase(A, x, y, q);
    if (!q.good) return;
    const long n = (long)y * A.W + x;
    finish(A, n, q, refine_global<DT>(A, n, q));
}

template <int TX, int TY, int DT>
__global__ void __launch_bounds__(TX * TY) fwd_kernel(EdgeArgs A, int remap) {
    const int tiles_x = (A.W + TX - 1) / TX, tiles = tiles_x * ((A.H + TY - 1) / TY);
    const int t = tile_of_block(blockIdx.x, tiles, remap != 0);
    if (t < 0) return;
    int x = (t % tiles_x) * TX + (int)(threadIdx.x % TX);
    int y = (t / tiles_x) * TY + (int)(threadIdx.x / TX);
    if (x >= A.W || y >= A.H) return;
    match_query<DT>(A, x, y);
}

// Minimum / maximum over the 64 lanes of a wave (every lane active), in every
// lane: DPP quad swaps, half-row and row mirrors give the 16-lane result in
// each row, then the four rows are combined from scalar registers.
template <bool MAX>
__device__ __forceinline__ int wave_extreme(int v) {
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false));  // row_mirror
    return op(op(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
              op(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ int wave_min(int v) { return wave_extreme<false>(v); }
__device__ __forceinline__ int wave_max(int v) { return wave_extreme<true>(v); }

// n / d for 0 <= n < 2^16 and 1 <= d < 2^16 with one 32-bit multiply-high:
// magic = ceil(2^32 / d), and the rounding excess n (magic d - 2^32) / 2^32
// stays below 1/d.  d = 1, whose magic 2^32 does not fit in 32 bits, is
// taken apart (a one-column window or region).
struct SmallDiv {
    uint32_t magic;
    bool one;
    __device__ __forceinline__ explicit SmallDiv(int d)
        : magic((uint32_t)((0x100000000ull + (unsigned long long)d - 1ull) / (unsigned long long)d)), one(d == 1) {}
    __device__ __forceinline__ int operator()(int n) const { return one ? n : (int)__umulhi((uint32_t)n, magic); }
};

// Bounding box (lx, hx, ly, hy) over the block: min / max of every lane's
// values (INT_MAX / INT_MIN for lanes without one).  Ends with a barrier.
template <int NT>
__device__ __forceinline__ void block_box(int& lx, int& hx, int& ly, int& hy, int* box) {
    const int tid = threadIdx.x;
    lx = wave_min(lx); hx = wave_max(hx); ly = wave_min(ly); hy = wave_max(hy);
    const int wv = tid >> 6;
    __syncthreads();  // earlier readers of box are done
    if ((tid & 63) == 0) { box[4 * wv] = lx; box[4 * wv + 1] = hx; box[4 * wv + 2] = ly; box[4 * wv + 3] = hy; }
    __syncthreads();
    lx = box[0]; hx = box[1]; ly = box[2]; hy = box[3];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) {
        lx = min(lx, box[4 * w]); hx = max(hx, box[4 * w + 1]);
        ly = min(ly, box[4 * w + 2]); hy = max(hy, box[4 * w + 3]);
    }
}

// Margin (pixels) of the staged ray window around the bilinear cells of the
// tile's queries: the default; the persistent kernel also comes with 1 and 3
// for the autotuner (samples outside the window read global memory, so the
// margin changes where values come from, never the values).
constexpr int kRayMargin = 2;

// Copies the ray records of window [lx, lx + rw) x [ly, ly + rh) into `lds`
// in the layout WindowRays reads (direct global -> LDS loads: planes P0 and P1
// of window pixel k at lds[2k] and lds[2k + 1], then plane Z, one float per
// pixel); the caller waits for them and synchronises.  Needs 36 rw rh bytes.
template <int NT>
__device__ __forceinline__ void stage_rays(const EdgeArgs& A, float4* lds, int lx, int ly, int rw, int rh) {
    const int tid = threadIdx.x;
    const int npx = rw * rh, slots = kRecP4 * npx;
    const SmallDiv div_rw(rw);
    for (int c0 = tid & ~63; c0 < slots; c0 += NT) {
        const int c = c0 + (tid & 63);
        if (c < slots) {
            const int pix = c >> 1, j = c & 1;
            const int ry = div_rw(pix), rx = pix - ry * rw;
            __builtin_amdgcn_global_load_lds(A.rays + (long)j * A.H * A.W + (long)(ly + ry) * A.W + lx + rx,
                                             (__attribute__((address_space(3))) void*)(lds + c0), 16, 0, 0);
        }
    }
    const float* z = reinterpret_cast<const float*>(A.rays + (long)kRecP4 * A.H * A.W);
    float* ldz = reinterpret_cast<float*>(lds + slots);
    for (int c0 = tid & ~63; c0 < npx; c0 += NT) {
        const int c = c0 + (tid & 63);
        if (c < npx) {
            const int ry = div_rw(c), rx = c - ry * rw;
            __builtin_amdgcn_global_load_lds(z + (long)(ly + ry) * A.W + lx + rx,
                                             (__attribute__((address_space(3))) void*)(ldz + c0), 4, 0, 0);
        }
    }
}

// Phase 1 of a tile with the ray records staged in LDS.  Queries that start on
// their own pixel (no p_init) sample the cells of the tile's pixels first, so
// the window of those cells (plus MARGIN) is staged before the query
// setup, with no dependence on it.  After the first LM iteration the window
// around the cells every query has reached (plus MARGIN) is staged
// unless the first window already holds it (at most cap_px pixels).  Samples
// outside the staged window read global memory.  All lanes of the block call
// this; [tx_lo, tx_hi] x [ty_lo, ty_hi] are the tile's pixels in the image.
// EARLY enables the first window: it shortens the latency of a launch with
// one wave of tiles and costs bandwidth in a persistent launch, whose other
// workgroups hide that latency anyway.
template <int NT, bool EARLY, int MARGIN = kRayMargin, int UNROLL = 1>
__device__ __forceinline__ void tile_lm(const EdgeArgs& A, int x, int y, bool inside, QState& q,
                                        float4* lds, int cap_px, int* box, int tx_lo, int tx_hi, int ty_lo,
                                        int ty_hi) {
    const int H = A.H, W = A.W;
    float3 t;
    LMState st;
    q.good = false;
    const GlobalRays g(A.rays, H, W);
    const int first = min(A.K, 1);
    int wx = 0, wy = 0, ww = 0, wh = 0;  // staged window (ww == 0: none)
    if (EARLY && !A.p_init) {
        const int lx = max(min(tx_lo, W - 2) - MARGIN, 0), hx = min(min(tx_hi, W - 2) + 1 + MARGIN, W - 1);
        const int ly = max(min(ty_lo, H - 2) - MARGIN, 0), hy = min(min(ty_hi, H - 2) + 1 + MARGIN, H - 1);
        if ((hx - lx + 1) * (hy - ly + 1) <= cap_px) {
            wx = lx; wy = ly; ww = hx - lx + 1; wh = hy - ly + 1;
            stage_rays<NT>(A, lds, wx, wy, ww, wh);
        }
    }
    const bool act = inside && lm_setup(A, x, y, q, t, st);
    if (ww) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (act) {
        if (ww) {
            const WindowRays wr{lds, wx, wy, ww, wh, g};
            lm_start(wr, H, W, A.lambda0, t, st);
            lm_iterate<UNROLL>(wr, H, W, t, first, st, A.K == first);
        } else {
            lm_start(g, H, W, A.lambda0, t, st);
            lm_iterate<UNROLL>(g, H, W, t, first, st, A.K == first);
        }
    }
    int lx = INT_MAX, hx = INT_MIN, ly = INT_MAX, hy = INT_MIN;
    if (act) {
        const int cx = min((int)floorf(st.px), W - 2), cy = min((int)floorf(st.py), H - 2);
        lx = max(cx - MARGIN, 0); hx = min(cx + 1 + MARGIN, W - 1);
        ly = max(cy - MARGIN, 0); hy = min(cy + 1 + MARGIN, H - 1);
    }
    block_box<NT>(lx, hx, ly, hy, box);  // ends with a barrier: no lane reads the window any more
    const int rw = hx - lx + 1, rh = hy - ly + 1;
    const bool more = A.K > first && hx >= lx;
    const bool held = ww && lx >= wx && hx < wx + ww && ly >= wy && hy < wy + wh;
    if (more && !held) {
        if (rw * rh <= cap_px) {
            wx = lx; wy = ly; ww = rw; wh = rh;
            stage_rays<NT>(A, lds, wx, wy, ww, wh);
            __builtin_amdgcn_s_waitcnt(0);
        } else {
            ww = 0;
            if (threadIdx.x == 0) count_path(kPathLmGlobal);
        }
    }
    __syncthreads();
    if (act) {
        if (more && ww) {
            const WindowRays wr{lds, wx, wy, ww, wh, g};
            lm_iterate<UNROLL>(wr, H, W, t, A.K - first, st);
        } else {
            lm_iterate<UNROLL>(g, H, W, t, A.K - first, st);
        }
        lm_finish(A, x, y, st, q);
    }
}

// Region pixels of the LDS refine: 832 px x 96 B = 78 KiB, two workgroups per CU.
constexpr int kRegionPx = 832;

// LDS needed by one tile of the LDS path.
struct TileLds {
    union {
        float4 desc[6 * kRegionPx];        // refine region (six planes)
        float4 rays[6 * kRegionPx];        // LM ray window (36-byte records of up to 2218 pixels)
    };
    int box[4 * 16];
};

// One TX x TY query tile with the LDS refine.  Every thread of the block
// calls this (threads outside the image skip the work but join the
// barriers).  The refine region is the bounding box of the windows of the
// tile's good queries; if it exceeds kRegionPx pixels the tile refines from
// global memory instead.
template <int TX, int TY>
__device__ __forceinline__ void tile_lds(const EdgeArgs& A, int tx, int ty, TileLds& S) {
    constexpr int NT = TX * TY;
    const int tid = threadIdx.x;
    const int x = tx * TX + tid % TX, y = ty * TY + tid / TX;
    const bool inside = x < A.W && y < A.H;
    QState q;
    tile_lm<NT, false>(A, x, y, inside, q, S.rays, (int)(sizeof(S.rays) / kRecBytes), S.box, tx * TX, min(tx * TX + TX, A.W) - 1, ty * TY,
                min(ty * TY + TY, A.H) - 1);
    const int r = A.r, W = A.W, H = A.H;
    int lx = INT_MAX, hx = INT_MIN, ly = INT_MAX, hy = INT_MIN;
    if (q.good) {
        int mx0 = round_half_up(q.px), my0 = round_half_up(q.py);
        lx = max(mx0 - r, 0); hx = min(mx0 + r, W - 1);
        ly = max(my0 - r, 0); hy = min(my0 + r, H - 1);
    }
    block_box<NT>(lx, hx, ly, hy, S.box);
    const int rw = hx - lx + 1, rh = hy - ly + 1;
    const bool any = hx >= lx;
    const bool use_lds = any && rw * rh <= kRegionPx && A.levels == 1;
    if (any && !use_lds && tid == 0) count_path(kPathRefineGlobal);
    if (use_lds) {
        // Direct global -> LDS loads (no registers, all in flight at once).  LDS
        // slot c = k * kRegionPx + pix holds float4 k of region pixel pix; each
        // wave fills 64 consecutive slots, lane i the slot base + i.
        constexpr int kSlots = 6 * kRegionPx;
        const float4* src4 = reinterpret_cast<const float4*>(A.Dii);
        const int np = rw * rh;
        const SmallDiv div_rw(rw);
        for (int c0 = tid & ~63; c0 < kSlots; c0 += NT) {
            const int c = c0 + (tid & 63);
            const int k = c / kRegionPx, pix = c - (c / kRegionPx) * kRegionPx;
            if (k < 6 && pix < np) {
                const int ry = div_rw(pix), rx = pix - ry * rw;
                __builtin_amdgcn_global_load_lds(src4 + ((long)(ly + ry) * W + lx + rx) * 6 + k,
                                                 (__attribute__((address_space(3))) void*)(S.desc + c0), 16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    if (q.good) {
        const long n = (long)y * W + x;
        long bi = use_lds ? refine_lds<kRegionPx>(A, n, q, S.desc, lx, ly, rw) : refine_global<24>(A, n, q);
        finish(A, n, q, bi);
    }
    __syncthreads();  // the next tile may overwrite S
}

// ---------------------------------------------------------------- fp16 pre-filtered refine
//
// Exact first-maximum refine with an fp16 pre-filter (D = 24, r <= 5).  The
// staged region holds D^i_i in fp16 (three planes of eight halves: 48 B per
// pixel), so one pass scores every window candidate with v_dot2_f32_f16.
// Both operands are scaled by 2^8 before the conversion (exact), which moves
// the fp16 subnormal range 2^8 below the values it would otherwise hold.
// Any candidate whose fp32 score could equal the fp32 maximum has a scaled
// fp16 score within tau of the running fp16 maximum, where tau bounds twice
// the sum of the fp16 error (conversion of both scaled operands with
// round-to-nearest, relative 2^-11, absolute 2^-14 for values that may flush,
// plus fp32 accumulation) and the fp32 error of the exact dot (24 u32 |q||d|),
// all in scaled units.  Those candidates are rescored exactly from global
// memory in row-major order with the same products and order as every other
// refine path, so the result is the same index.

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

constexpr int kRegionPx16 = 832;          // 832 px x 48 B = 39 KiB: four workgroups per CU
constexpr int kRegionPx16Multi = 1088;    // the multi-level kernel: 51 KiB, three workgroups per CU
constexpr int kRegionPx16Small = 256;     // 8 x 8 tiles: 12 KiB, twelve one-wave workgroups per CU

// Region capacity (pixels) of a tile shape's fp16 LDS buffers.
template <int TX, int TY, bool MULTI>
constexpr int f16_cap() {
    return MULTI ? kRegionPx16Multi : (TX * TY <= 64 ? kRegionPx16Small : kRegionPx16);
}
constexpr float kF16Max = 60000.f;        // larger scaled magnitudes fall back to the exact scan
constexpr float kScale16 = 256.f;         // 2^8, applied to both operands before the conversion
constexpr float kU16 = 4.8828125e-4f;     // 2^-11
constexpr float kU32x24 = 1.4305115e-6f;  // 24 * 2^-24
constexpr float kFlush16 = 6.1035156e-5f; // 2^-14
constexpr float kSqrt24Up = 4.8989797f;   // sqrt(24) rounded up

template <int CAP>
struct TileLds16 {
    union {
        uint4 desc[3 * CAP];               // refine region (three fp16 planes of CAP pixels)
        float4 rays[3 * CAP];              // LM ray window (36-byte records of up to 4 CAP / 3 pixels)
    };
    int box[4 * 16];
    float stat[16];                       // per wave: largest |d|^2 of a region pixel
};

__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
    h2_t v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float dot16(const uint32_t* q16, uint4 a, uint4 b, uint4 c) {
    float acc = 0.f;
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[0]), __builtin_bit_cast(h2_t, a.x), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[1]), __builtin_bit_cast(h2_t, a.y), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[2]), __builtin_bit_cast(h2_t, a.z), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[3]), __builtin_bit_cast(h2_t, a.w), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[4]), __builtin_bit_cast(h2_t, b.x), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[5]), __builtin_bit_cast(h2_t, b.y), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[6]), __builtin_bit_cast(h2_t, b.z), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[7]), __builtin_bit_cast(h2_t, b.w), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[8]), __builtin_bit_cast(h2_t, c.x), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[9]), __builtin_bit_cast(h2_t, c.y), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[10]), __builtin_bit_cast(h2_t, c.z), acc, false);
    acc = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, q16[11]), __builtin_bit_cast(h2_t, c.w), acc, false);
    return acc;
}

// Exact fp32 score of reference pixel m, same products and order as QueryDesc<24>::dot.
__device__ __forceinline__ float exact24(const float* __restrict__ q, const float* __restrict__ Dii, long m) {
    const float4* s = reinterpret_cast<const float4*>(Dii + 24 * m);
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float4 v = s[k];
        acc = fmaf(q[4 * k], v.x, acc);
        acc = fmaf(q[4 * k + 1], v.y, acc);
        acc = fmaf(q[4 * k + 2], v.z, acc);
        acc = fmaf(q[4 * k + 3], v.w, acc);
    }
    return acc;
}

// Pass 1 over a window that lies inside the image, for a radius R and a
// candidate spacing SP fixed at compile time: the candidates of a row are unrolled (LDS addresses are the
// row base plus immediate offsets), the row's scores are kept in registers,
// the running maximum takes the row's maximum, and each candidate of the row
// survives if its score is within tau of that running maximum.  A candidate
// that survives against the final maximum survives against any earlier one,
// so no candidate that can be the exact maximum is dropped.  The survivor
// bits are shifted into a 128-bit word hi:lo, leaving candidate j of the
// window on bit N - 1 - j; a bit reversal then gives the row-major masks of
// the generic pass (candidate j on bit j).  w: LDS record of the window's
// top-left candidate.
template <int R, int SP, int CAP>
__device__ __forceinline__ void scan16_inside(const uint32_t* q16, const uint4* __restrict__ w, int rw, float tau,
                                              float& run, uint64_t& mask0, uint64_t& mask1) {
    constexpr int S = 2 * R + 1, N = S * S;
    static_assert(N <= 128 && S < 32, "mask width");
    if constexpr (N <= 64) {
        // The whole mask in one word: candidate (dy, dx) at bit dy * S + dx,
        // the row-major order the survivor pass pops in (bit values 1 .. 2^(S-1)
        // are inline constants).
        uint64_t m = 0;
#pragma unroll 1
        for (int dy = 0; dy < S; ++dy, w += SP * rw) {
            float sc[S];
#pragma unroll
            for (int dx = 0; dx < S; ++dx)
                sc[dx] = dot16(q16, w[SP * dx], w[SP * dx + CAP], w[SP * dx + 2 * CAP]);
            float rm = sc[0];
#pragma unroll
            for (int dx = 1; dx < S; ++dx) rm = fmaxf(rm, sc[dx]);
            run = fmaxf(run, rm);
            const float thr = run - tau;
            uint32_t rb = 0;
#pragma unroll
            for (int dx = 0; dx < S; ++dx) rb |= sc[dx] >= thr ? (1u << dx) : 0u;
            m |= (uint64_t)rb << (dy * S);
        }
        mask0 = m;
        mask1 = 0;
        return;
    }
    uint64_t lo = 0, hi = 0;
#pragma unroll 1
    for (int dy = 0; dy < S; ++dy, w += SP * rw) {
        float sc[S];
#pragma unroll
        for (int dx = 0; dx < S; ++dx)
            sc[dx] = dot16(q16, w[SP * dx], w[SP * dx + CAP], w[SP * dx + 2 * CAP]);
        float rm = sc[0];
#pragma unroll
        for (int dx = 1; dx < S; ++dx) rm = fmaxf(rm, sc[dx]);
        run = fmaxf(run, rm);
        const float thr = run - tau;
        uint32_t rb = 0;
#pragma unroll
        for (int dx = 0; dx < S; ++dx) rb = rb + rb + (sc[dx] >= thr ? 1u : 0u);
        hi = (hi << S) | (lo >> (64 - S));
        lo = (lo << S) | rb;
    }
    const uint64_t rhi = __builtin_bitreverse64(lo), rlo = __builtin_bitreverse64(hi);
    constexpr int sh = 128 - N;  // forward mask = (rhi:rlo) >> sh
    if constexpr (sh >= 64) {
        mask0 = rhi >> (sh - 64);
        mask1 = 0;
    } else {
        mask0 = (rlo >> sh) | (rhi << (64 - sh));
        mask1 = rhi >> sh;
    }
}

// A query descriptor for the fp16 pre-filter: fp32 elements (exact rescoring),
// the scaled fp16 copy, and the bounds of the error budget (scaled units).
struct Query16 {
    QueryDesc<24> qd;
    uint32_t q16[12];
    float qn, ql1;   // bounds on |q| and |q|_1 (times kScale16)
    bool ok;         // |q| within the fp16 range
};

__device__ __forceinline__ void load_query16(const EdgeArgs& A, long n, Query16& Q) {
    Q.qd.load(A.Dji, n, 24);
    // |q_k| <= |q| bounds every element (fp16 range) and |q|_1 <= sqrt(24) |q|;
    // the 1.0001 margin covers the rounding of the fp32 norm.
    float qn2 = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) qn2 = fmaf(Q.qd.q[k], Q.qd.q[k], qn2);
    Q.qn = sqrtf(qn2) * 1.0001f * kScale16;
    Q.ok = Q.qn <= kF16Max;
    Q.ql1 = kSqrt24Up * Q.qn;
#pragma unroll
    for (int k = 0; k < 12; ++k) Q.q16[k] = pack_h2(Q.qd.q[2 * k] * kScale16, Q.qd.q[2 * k + 1] * kScale16);
}

// Survivor threshold tau of the fp16 pre-filter in scaled units (both
// operands times kScale16): twice the bound on the fp16 score's error plus
// that of the exact fp32 rescoring.  dnorm: bound on |d| over the staged
// region, dl1: bound on |d|_1.
__device__ __forceinline__ float f16_tau(const Query16& Q, float dnorm, float dl1) {
    const float qn = Q.qn;
    dnorm *= kScale16;
    dl1 *= kScale16;
    const float eps16 = (2.f * kU16 + kU16 * kU16 + kU32x24) * qn * dnorm + kFlush16 * (Q.ql1 + dl1);
    const float eps32 = kU32x24 * qn * dnorm;
    return 2.f * (eps16 + eps32) * 1.0001f + 1e-30f;
}

// Pass 2 of the fp16 refine: exact scores of the survivors (candidate k of the
// (2r+1)^2 window on bit k of mask1:mask0) in row-major order, two per step
// so that both descriptor reads are in flight together; the first maximum.
__device__ __forceinline__ long f16_rescore(const EdgeArgs& A, const Query16& Q, int mx0, int my0, int sp,
                                            uint64_t mask0, uint64_t mask1) {
    const int W = A.W, r = A.r, side = 2 * r + 1;
    auto pop = [&](uint64_t& m0, uint64_t& m1) -> int {
        if (m0) { const int k = __builtin_ctzll(m0); m0 &= m0 - 1; return k; }
        if (m1) { const int k = 64 + __builtin_ctzll(m1); m1 &= m1 - 1; return k; }
        return -1;
    };
    auto pixel = [&](int kk) -> long {
        const int dy = kk / side, dx = kk - dy * side;
        return (long)(my0 + sp * (dy - r)) * W + (mx0 + sp * (dx - r));
    };
    float best = -INFINITY;
    long bi = -1;
    while (mask0 | mask1) {
        const int k1 = pop(mask0, mask1), k2 = pop(mask0, mask1);
        const long m1 = pixel(k1), m2 = k2 >= 0 ? pixel(k2) : m1;
        const float s1 = exact24(Q.qd.q, A.Dii, m1), s2 = exact24(Q.qd.q, A.Dii, m2);
        if (s1 > best) { best = s1; bi = m1; }
        if (k2 >= 0 && s2 > best) { best = s2; bi = m2; }
    }
    return bi;
}

// Pass 1 of the fp16 refine over the window rows that lie in one band of a
// region staged band by band: region rows [ry0, bhi] (inside the image) are in
// LDS, ry0 first.  The running maximum `run` and the survivor masks carry over
// from the bands above, so the candidates are still thresholded in row-major
// order, each against the largest score before it; tau only grows from band
// to band (it follows the largest |d| staged so far), so every survivor test
// keeps the margin that the candidates scanned until then need.
template <int CAP>
__device__ __forceinline__ void f16_scan_band(const EdgeArgs& A, const Query16& Q, int mx0, int my0, int sp,
                                              const uint4* __restrict__ sd, int rx0, int ry0, int rw, int bhi,
                                              float tau, float& run, uint64_t& mask0, uint64_t& mask1) {
    const int W = A.W, r = A.r, side = 2 * r + 1;
    for (int dy = -r; dy <= r; ++dy) {
        const int my = my0 + sp * dy;
        if (my < ry0 || my > bhi) continue;
        const uint4* d = sd + (my - ry0) * rw - rx0;
        for (int dx = -r; dx <= r; ++dx) {
            const int mx = mx0 + sp * dx;
            if (mx < 0 || mx >= W) continue;
            const int k = (dy + r) * side + (dx + r);
            const float s16 = dot16(Q.q16, d[mx], d[mx + CAP], d[mx + 2 * CAP]);
            run = __builtin_amdgcn_fmed3f(s16, run, INFINITY);
            if (s16 >= run - tau) {
                if (k < 64) mask0 |= 1ull << k; else mask1 |= 1ull << (k - 64);
            }
        }
    }
}

// One level of the exact first-maximum refine with the fp16 pre-filter: the
// (2r+1)^2 grid of spacing sp around (mx0, my0), over a staged region that
// holds every candidate inside the image.  dnorm: bound on |d| over the
// region, dl1: bound on |d|_1.
template <int CAP>
__device__ __forceinline__ long refine_f16_level(const EdgeArgs& A, const Query16& Q, int mx0, int my0, int sp,
                                                 const uint4* __restrict__ sd, int rx0, int ry0, int rw, float dnorm,
                                                 float dl1) {
    const int H = A.H, W = A.W, r = A.r, side = 2 * r + 1;
    const float tau = f16_tau(Q, dnorm, dl1);

    // Pass 1: fp16 scores in row-major window order over the candidates
    // inside the image; the running maximum is seeded with the window centre
    // (v_med3 against +inf is the maximum of two non-NaN scores).
    const uint4* c0 = sd + (my0 - ry0) * rw + (mx0 - rx0);
    float run = dot16(Q.q16, c0[0], c0[CAP], c0[2 * CAP]);
    uint64_t mask0 = 0, mask1 = 0;
    const int reach = r * sp;
    // Wave-uniform choice: the unrolled scan when every active lane's window
    // lies inside the image, the bounded loop otherwise.
    const bool whole = mx0 - reach >= 0 && mx0 + reach <= W - 1 && my0 - reach >= 0 && my0 + reach <= H - 1;
    const uint4* w = sd + (my0 - reach - ry0) * rw + (mx0 - reach - rx0);
    const bool all_whole = __all(whole) != 0;
    if (all_whole && sp == 1 && r == 3) {
        scan16_inside<3, 1, CAP>(Q.q16, w, rw, tau, run, mask0, mask1);
    } else if (all_whole && sp == 1 && r == 2) {
        scan16_inside<2, 1, CAP>(Q.q16, w, rw, tau, run, mask0, mask1);
    } else if (all_whole && sp == 1 && r == 4) {
        scan16_inside<4, 1, CAP>(Q.q16, w, rw, tau, run, mask0, mask1);
    } else if (all_whole && sp == 2 && r == 3) {
        scan16_inside<3, 2, CAP>(Q.q16, w, rw, tau, run, mask0, mask1);
    } else {
        for (int dy = -r; dy <= r; ++dy) {
            const int my = my0 + sp * dy;
            if (my < 0 || my >= H) continue;
            const uint4* d = sd + (my - ry0) * rw - rx0;
            for (int dx = -r; dx <= r; ++dx) {
                const int mx = mx0 + sp * dx;
                if (mx < 0 || mx >= W) continue;
                const int k = (dy + r) * side + (dx + r);
                const float s16 = dot16(Q.q16, d[mx], d[mx + CAP], d[mx + 2 * CAP]);
                run = __builtin_amdgcn_fmed3f(s16, run, INFINITY);
                if (s16 >= run - tau) {
                    if (k < 64) mask0 |= 1ull << k; else mask1 |= 1ull << (k - 64);
                }
            }
        }
    }
    // Pass 2: exact scores of the survivors.
    return f16_rescore(A, Q, mx0, my0, sp, mask0, mask1);
}

// Stages region rows [ly, ly + rh) x columns [lx, lx + rw) of D^i_i into the
// three fp16 planes of `desc` (region pixel pix of plane k at desc[k * CAP +
// pix], scaled by kScale16): each lane converts whole pixels (six float4
// loads, the norm, three fp16 planes), kBatch pixels per step with all loads
// issued before the conversions and stores.  Returns the lane's largest |d|^2
// (+inf for a pixel with a non-finite element or squares that overflow, which
// fails the caller's range test).
template <int NT, int CAP, int kBatch>
__device__ __forceinline__ float stage_region16(const EdgeArgs& A, uint4* desc, int lx, int ly, int rw, int rh) {
    const int tid = threadIdx.x, W = A.W;
    const float4* src4 = reinterpret_cast<const float4*>(A.Dii);
    const int total = rw * rh;
    const SmallDiv div_rw(rw);
    float pn2 = 0.f;
    for (int p00 = 0; p00 < total; p00 += kBatch * NT) {
        float4 v[kBatch][6];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int pix = p00 + tid + i * NT;
            if (pix < total) {
                const int ry = div_rw(pix), rx = pix - ry * rw;
                const float4* src = src4 + ((long)(ly + ry) * W + lx + rx) * 6;
#pragma unroll
                for (int k = 0; k < 6; ++k) v[i][k] = src[k];
            }
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int pix = p00 + tid + i * NT;
            if (pix < total) {
                float e2 = 0.f;
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    e2 += v[i][k].x * v[i][k].x + v[i][k].y * v[i][k].y + v[i][k].z * v[i][k].z + v[i][k].w * v[i][k].w;
                pn2 = fmaxf(pn2, isfinite(e2) ? e2 : INFINITY);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float4 u = v[i][2 * k], w = v[i][2 * k + 1];
                    desc[k * CAP + pix] =
                        make_uint4(pack_h2(u.x * kScale16, u.y * kScale16), pack_h2(u.z * kScale16, u.w * kScale16),
                                   pack_h2(w.x * kScale16, w.y * kScale16), pack_h2(w.z * kScale16, w.w * kScale16));
                }
            }
        }
    }
    return pn2;
}

// Largest pn2 over the block (ends with a barrier, so the staged region is
// complete).  Region bounds: |d| <= sqrt(pn2) for every pixel, so every
// element |d_k| <= sqrt(pn2) (kScale16^2 pn2 <= kF16Max^2 keeps the scaled
// conversion finite), and |d|_1 <= sqrt(24) |d| (Cauchy-Schwarz).
template <int NT>
__device__ __forceinline__ float block_max16(float pn2, float* stat) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pn2 = fmaxf(pn2, __shfl_xor(pn2, o, 64));
    if ((tid & 63) == 0) stat[tid >> 6] = pn2;
    __syncthreads();
    pn2 = stat[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) pn2 = fmaxf(pn2, stat[w]);
    return pn2;
}

// Bands of whole region rows that the multi-level kernel stages and scans one
// after another when a level's region exceeds LDS (more fall back to the exact
// global scan).
constexpr int kMaxBands = 6;

// One TX x TY tile with the fp16 pre-filtered refine, level by level for the
// coarse-to-fine refine when MULTI is set (level l scans the grid of spacing 2^l around the
// previous level's best).  For each level the region is the bounding box of
// the windows of the tile's good queries.  With MULTI set, a region that does
// not fit LDS is staged and pre-filtered in bands of whole rows (at most
// kMaxBands).  A level whose region does not fit (in bands), whose radius
// exceeds 5, or whose region holds a value too large for fp16 is scanned
// exactly from global memory instead (the whole tile at that level).
template <int TX, int TY, bool EARLY, int MARGIN = kRayMargin, int UNROLL = 1, bool MULTI = false>
__device__ __forceinline__ void tile_f16(const EdgeArgs& A, int tx, int ty, TileLds16<f16_cap<TX, TY, MULTI>()>& S) {
    constexpr int NT = TX * TY;
    constexpr int CAP = f16_cap<TX, TY, MULTI>();
    const int tid = threadIdx.x;
    const int x = tx * TX + tid % TX, y = ty * TY + tid / TX;
    const bool inside = x < A.W && y < A.H;
    QState q;
    tile_lm<NT, EARLY, MARGIN, UNROLL>(A, x, y, inside, q, S.rays, (int)(sizeof(S.rays) / kRecBytes), S.box, tx * TX, min(tx * TX + TX, A.W) - 1, ty * TY,
                min(ty * TY + TY, A.H) - 1);
    const int r = A.r, W = A.W, H = A.H;
    const long n = (long)y * W + x;
    long bi = -1;
    bool live = q.good;   // takes part in the level below
    int cx = live ? round_half_up(q.px) : 0, cy = live ? round_half_up(q.py) : 0;
    // MULTI = false: one level (the launcher takes the MULTI kernel for L > 1;
    // a constant trip count keeps the single-level kernel free of spills).
    Query16 Q;            // read once, at the first level that needs it
    bool have_q = false;
    for (int lev = MULTI ? A.levels - 1 : 0; lev >= 0; --lev) {
        const int sp = 1 << lev, reach = r * sp;
        int lx = INT_MAX, hx = INT_MIN, ly = INT_MAX, hy = INT_MIN;
        if (live) {
            lx = max(cx - reach, 0); hx = min(cx + reach, W - 1);
            ly = max(cy - reach, 0); hy = min(cy + reach, H - 1);
        }
        block_box<NT>(lx, hx, ly, hy, S.box);  // ends with a barrier: the previous level is done with S
        const int rw = hx - lx + 1, rh = hy - ly + 1;
        const bool any = hx >= lx;
        // The query descriptor is read once, after the first level's region (or
        // its first band) is staged, so that its registers are not live during
        // that staging; the later levels of the multi-level kernel keep it.  A
        // query whose own descriptor is outside the fp16 range refines every
        // level exactly from global memory and leaves the levels below.
        auto query = [&]() {
            if (have_q) return;
            have_q = true;
            load_query16(A, n, Q);
            if (!Q.ok) {
                count_path(kPathRefineQuery);
                bi = refine_global<24>(A, n, q);
                live = false;
            }
        };
        long lb = -1;
        // Rows per band when the multi-level kernel stages a region that
        // exceeds LDS band by band (0: not banded).
        int band = 0;
        if constexpr (MULTI) {
            if (any && r <= 5 && rw * rh > CAP && rw <= CAP && rh <= kMaxBands * (CAP / rw)) band = CAP / rw;
        }
        if (band > 0) {
            if (tid == 0) count_path(kPathRefineBands);
            float pn2 = 0.f, run = -INFINITY;
            uint64_t mask0 = 0, mask1 = 0;
            bool ok16 = true;
            for (int b0 = 0; b0 < rh; b0 += band) {
                const int nr = min(band, rh - b0);
                if (b0 > 0) __syncthreads();  // every lane is done with the previous band
                pn2 = fmaxf(pn2, block_max16<NT>(stage_region16<NT, CAP, 1>(A, S.desc, lx, ly + b0, rw, nr), S.stat));
                if (!(pn2 <= (kF16Max / kScale16) * (kF16Max / kScale16))) {
                    ok16 = false;  // the same for every lane
                    break;
                }
                if (live) query();
                if (live) {
                    const float dnorm = sqrtf(pn2) * 1.0001f;
                    f16_scan_band<CAP>(A, Q, cx, cy, sp, S.desc, lx, ly + b0, rw, ly + b0 + nr - 1,
                                       f16_tau(Q, dnorm, kSqrt24Up * dnorm), run, mask0, mask1);
                }
            }
            if (!ok16 && tid == 0) count_path(kPathRefineGlobal);
            if (live) query();
            if (live)
                lb = ok16 ? f16_rescore(A, Q, cx, cy, sp, mask0, mask1) : refine_global_level<24>(A, Q.qd, cx, cy, sp);
        } else {
            bool use16 = any && rw * rh <= CAP && r <= 5;
            float pn2 = 0.f;  // largest |d|^2 over the region's pixels
            if (use16) pn2 = stage_region16<NT, CAP, 2>(A, S.desc, lx, ly, rw, rh);
            pn2 = block_max16<NT>(pn2, S.stat);
            use16 = use16 && pn2 <= (kF16Max / kScale16) * (kF16Max / kScale16);
            if (any && !use16 && tid == 0) count_path(kPathRefineGlobal);
            if (live) query();
            if (live) {
                const float dnorm = sqrtf(pn2) * 1.0001f;
                lb = use16 ? refine_f16_level<CAP>(A, Q, cx, cy, sp, S.desc, lx, ly, rw, dnorm, kSqrt24Up * dnorm)
                           : refine_global_level<24>(A, Q.qd, cx, cy, sp);
            }
        }
        if (live) {
            if (lb < 0) {
                live = false;
            } else {
                bi = lb;
                cx = (int)(lb % W);
                cy = (int)(lb / W);
            }
        }
    }
    if (q.good) finish(A, n, q, bi);
    __syncthreads();  // the next tile may overwrite S
}

// Four workgroups of 256 lanes fit a CU by LDS; keep the registers within that too.
// The multi-level refine keeps more state per lane: three waves per SIMD.
template <int TX, int TY, bool MULTI>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(MULTI ? 3 : 4)))
fwd_f16_kernel(EdgeArgs A, int remap) {
    __shared__ TileLds16<f16_cap<TX, TY, MULTI>()> S;
    const int tiles_x = (A.W + TX - 1) / TX, tiles = tiles_x * ((A.H + TY - 1) / TY);
    const int t = tile_of_block(blockIdx.x, tiles, remap != 0);
    if (t < 0) return;
    tile_f16<TX, TY, true, kRayMargin, 1, MULTI>(A, t % tiles_x, t / tiles_x, S);
}

template <int TX, int TY>
__global__ void __launch_bounds__(TX * TY) fwd_lds_kernel(EdgeArgs A, int remap) {
    __shared__ TileLds S;
    const int tiles_x = (A.W + TX - 1) / TX, tiles = tiles_x * ((A.H + TY - 1) / TY);
    const int t = tile_of_block(blockIdx.x, tiles, remap != 0);
    if (t < 0) return;
    tile_lds<TX, TY>(A, t % tiles_x, t / tiles_x, S);
}

// ---------------------------------------------------------------- batched

// Edge of a global tile id: the last edge whose tile_begin <= tile.
__device__ __forceinline__ int find_edge(const EdgeArgs* __restrict__ E, int n_edges, int tile) {
    int lo = 0, hi = n_edges - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (E[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Prep tiles of edge e start at prep_begin[e] (prep_tiles(H, W) per edge).
// Also resets the forward's work-queue counter (the forward launch follows in
// the stream).
__global__ void __launch_bounds__(256) batched_prep_kernel(const EdgeArgs* __restrict__ E, const int32_t* __restrict__ prep_begin,
                                                           int n_edges, int32_t* __restrict__ counter) {
    __shared__ PrepLds S;
    int blk = blockIdx.x;
    if (blk == 0 && threadIdx.x == 0) counter[0] = 0;
    int lo = 0, hi = n_edges - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prep_begin[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    const EdgeArgs& A = E[lo];
    prep_tile(A.Xii, const_cast<float4*>(A.rays), A.H, A.W, blk - prep_begin[lo], S);
}

// Persistent forward over all edges: workgroups pop tile ids from a counter
// until none is left (every workgroup exits once the counter passes the last
// tile).  LDS tiles need D = 24 and 16-byte aligned descriptors on every edge.
// MODE 0: refine from global memory; 1: fp32 region in LDS; 2: fp16 pre-filter
// with ray-window margin MARGIN and LM unroll UNROLL.
template <int TX, int TY, int DT, int MODE, int MARGIN = kRayMargin, int UNROLL = 1, bool MULTI = false>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(MODE == 2 ? (MULTI ? 3 : 4) : 1)))
batched_fwd_kernel(const EdgeArgs* __restrict__ E, int n_edges, int total_tiles,
                                                               int32_t* __restrict__ counter) {
    __shared__ int s_tile;
    __shared__ typename std::conditional<
        MODE == 1, TileLds,
        typename std::conditional<MODE == 2, TileLds16<f16_cap<TX, TY, MULTI>()>, int>::type>::type S;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        int tile = s_tile;
        __syncthreads();
        if (tile >= total_tiles) return;
        int e = find_edge(E, n_edges, tile);
        const EdgeArgs A = E[e];
        int local = tile - A.tile_begin;
        int ty = local / A.tiles_x, tx = local - ty * A.tiles_x;
        if constexpr (MODE == 1) {
            tile_lds<TX, TY>(A, tx, ty, S);
        } else if constexpr (MODE == 2) {
            tile_f16<TX, TY, false, MARGIN, UNROLL, MULTI>(A, tx, ty, S);
        } else {
            int x = tx * TX + (int)(threadIdx.x % TX);
            int y = ty * TY + (int)(threadIdx.x / TX);
            if (x < A.W && y < A.H) match_query<DT>(A, x, y);
        }
    }
}


// ---------------------------------------------------------------- backward

// Zeroes a[0, count): scalar stores up to the first 16-byte boundary and after
// the last one, float4 stores in between.
__global__ void __launch_bounds__(256) fill_zero_kernel(float* __restrict__ a, long count) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    const long head = min(count, (long)(((16u - ((uint32_t)(uintptr_t)a & 15u)) & 15u) >> 2));
    if (i < head) a[i] = 0.f;
    float4* __restrict__ b = reinterpret_cast<float4*>(a + head);
    const long nb = (count - head) >> 2;
    for (long j = i; j < nb; j += stride) store_nt(b + j, make_float4(0.f, 0.f, 0.f, 0.f));
    const long t = head + (nb << 2) + i;
    if (t < count && i < 4) a[t] = 0.f;
}

// v -> N(X) v = (v - u (u.v)) / |X| with u = X/|X| (Supp. A, Eq. norm_jac).
__device__ __forceinline__ float3 norm_jac_apply(float3 X, float3 v) {
    float inv = rsq(X.x * X.x + X.y * X.y + X.z * X.z);
    float3 u = f3(X.x * inv, X.y * inv, X.z * inv);
    float uv = u.x * v.x + u.y * v.y + u.z * v.z;
    return f3((v.x - u.x * uv) * inv, (v.y - u.y * uv) * inv, (v.z - u.z * uv) * inv);
}

// Per-query inputs of the backward, read before the query's validity is
// known so that every load of a tile is in flight at once.
struct BwdQueryIn {
    float px, py, gp0, gp1;
    float3 gx, xq;  // grad_xhat[n] (zero without it), X^j_i[n]
};

// Loads and atomics through global (not flat) instructions: the pointers of
// an edge table read from memory are generic, which makes the compiler emit
// flat accesses that also count against the LDS wait counter.
template <class T>
__device__ __forceinline__ T ld_global(const T* ptr, long i) {
    return ((const __attribute__((address_space(1))) T*)ptr)[i];
}
__device__ __forceinline__ float3 ld_global_point(const float* X, long m) {
    return f3(ld_global(X, 3 * m), ld_global(X, 3 * m + 1), ld_global(X, 3 * m + 2));
}
__device__ __forceinline__ void add_global(float* ptr, float v) {
    __builtin_amdgcn_global_atomic_fadd_f32((__attribute__((address_space(1))) float*)ptr, v);
}

// Adjoint of one valid query: returns dXji[n] and the four corner pixels of p*
// with the gradient each receives in dXii (zero weight: none).
__device__ __forceinline__ float3 bwd_query(int H, int W, const float* __restrict__ Xii, bool has_gx,
                                            const BwdQueryIn& in, long cm[4], float3 gc[4], int& cx0, int& cy0) {
    const float px = in.px, py = in.py;
    int x0 = min(max((int)floorf(px), 0), W - 2), y0 = min(max((int)floorf(py), 0), H - 2);
    float a = px - (float)x0, b = py - (float)y0;
    const long cm_[4] = {(long)y0 * W + x0, (long)y0 * W + x0 + 1, (long)(y0 + 1) * W + x0, (long)(y0 + 1) * W + x0 + 1};
    float w[4] = {(1.f - a) * (1.f - b), a * (1.f - b), (1.f - a) * b, a * b};
    float3 X[4], R[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        X[c] = ld_global_point(Xii, cm_[c]);
        R[c] = unit_ray(X[c]);
    }
    float3 r = f3(w[0] * R[0].x + w[1] * R[1].x + w[2] * R[2].x + w[3] * R[3].x,
                  w[0] * R[0].y + w[1] * R[1].y + w[2] * R[2].y + w[3] * R[3].y,
                  w[0] * R[0].z + w[1] * R[1].z + w[2] * R[2].z + w[3] * R[3].z);
    // Exact derivatives of the bilinear ray sample.
    float3 drx = f3((1.f - b) * (R[1].x - R[0].x) + b * (R[3].x - R[2].x),
                    (1.f - b) * (R[1].y - R[0].y) + b * (R[3].y - R[2].y),
                    (1.f - b) * (R[1].z - R[0].z) + b * (R[3].z - R[2].z));
    float3 dry = f3((1.f - a) * (R[2].x - R[0].x) + a * (R[3].x - R[1].x),
                    (1.f - a) * (R[2].y - R[0].y) + a * (R[3].y - R[1].y),
                    (1.f - a) * (R[2].z - R[0].z) + a * (R[3].z - R[1].z));
    float3 j0 = norm_jac_apply(r, drx), j1 = norm_jac_apply(r, dry);

    float gp0 = in.gp0, gp1 = in.gp1;
    const float3 gx = in.gx;
    if (has_gx) {
        float3 dxx = f3((1.f - b) * (X[1].x - X[0].x) + b * (X[3].x - X[2].x),
                        (1.f - b) * (X[1].y - X[0].y) + b * (X[3].y - X[2].y),
                        (1.f - b) * (X[1].z - X[0].z) + b * (X[3].z - X[2].z));
        float3 dxy = f3((1.f - a) * (X[2].x - X[0].x) + a * (X[3].x - X[1].x),
                        (1.f - a) * (X[2].y - X[0].y) + a * (X[3].y - X[1].y),
                        (1.f - a) * (X[2].z - X[0].z) + a * (X[3].z - X[1].z));
        gp0 += dxx.x * gx.x + dxx.y * gx.y + dxx.z * gx.z;
        gp1 += dxy.x * gx.x + dxy.y * gx.y + dxy.z * gx.z;
    }
    float a00 = j0.x * j0.x + j0.y * j0.y + j0.z * j0.z;
    float a01 = j0.x * j1.x + j0.y * j1.y + j0.z * j1.z;
    float a11 = j1.x * j1.x + j1.y * j1.y + j1.z * j1.z;
    // A coordinate of p* on the image bound is held by the forward and does not
    // move; the other one is solved alone (both held: nothing moves).
    bool held_x = px <= 0.f || px >= (float)(W - 1);
    bool held_y = py <= 0.f || py >= (float)(H - 1);
    float mu0, mu1;
    bool solve;
    if (held_x && held_y) {
        solve = true;
        mu0 = mu1 = 0.f;
    } else if (held_x) {
        solve = a11 > 0.f;
        mu0 = 0.f;
        mu1 = solve ? gp1 * rcp(a11) : 0.f;
    } else if (held_y) {
        solve = a00 > 0.f;
        mu1 = 0.f;
        mu0 = solve ? gp0 * rcp(a00) : 0.f;
    } else {
        float det = a00 * a11 - a01 * a01;
        solve = det > 0.f && isfinite(det);
        float idet = solve ? rcp(det) : 0.f;
        mu0 = (a11 * gp0 - a01 * gp1) * idet;
        mu1 = (a00 * gp1 - a01 * gp0) * idet;
    }
    float3 v = f3(j0.x * mu0 + j1.x * mu1, j0.y * mu0 + j1.y * mu1, j0.z * mu0 + j1.z * mu1);
    const float3 dq = solve ? norm_jac_apply(in.xq, v) : f3(0.f, 0.f, 0.f);
    float irn = rsq(r.x * r.x + r.y * r.y + r.z * r.z);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float3 g = f3(w[c] * gx.x, w[c] * gx.y, w[c] * gx.z);
        bool has_ray = R[c].x != 0.f || R[c].y != 0.f || R[c].z != 0.f;
        if (w[c] != 0.f && solve && has_ray) {
            float3 nv = norm_jac_apply(X[c], v);
            float s = w[c] * irn;
            g.x -= s * nv.x; g.y -= s * nv.y; g.z -= s * nv.z;
        }
        cm[c] = w[c] == 0.f ? -1 : cm_[c];
        gc[c] = g;
    }
    cx0 = x0;
    cy0 = y0;
    return dq;
}

// Largest box of corner pixels a tile accumulates in LDS (24 B per pixel).
constexpr int kBwdLdsPx = 768;
// Plane stride (in 64-bit words) of the planar accumulator: five words past
// the window, so the three components of a pixel sit in different LDS banks.
constexpr int kBwdPlane = kBwdLdsPx + 5;
// Accumulator words, rounded up to whole 16-byte stores for the clear.
constexpr int kBwdAccWords = (3 * kBwdPlane + 1) & ~1;

// The tile's window in LDS sums signed 64-bit fixed-point numbers with integer
// atomics: LDS float atomics run at a fraction of the integer rate on this
// chip, and integer sums do not depend on the order of the additions.  The
// scale 2^S is set per tile from the largest |g| of its corner gradients,
// g_max < 2^(E+1) with E its unbiased exponent: S = 49 - E, so one term is
// below 2^50 and a pixel's sum of at most 256 terms (one per query of the
// tile) stays below 2^58.  A term is |v| 2^S rounded to the nearest integer,
// an error of at most 2^-(S+1) = 2^(E-50), about 2^-50 of g_max (subnormal
// terms included: fp32 -> fp64 and the power-of-two scale are exact).  The
// rounding adds 1.5 * 2^52: a double in [2^52, 2^53) has unit spacing, so the
// sum rounds to an integer that its low bits hold; subtracting the bit
// pattern of 1.5 * 2^52 leaves that integer (|v| 2^S < 2^51 is needed).
__device__ __forceinline__ long long bwd_to_fixed(float v, double scale) {
    const double t = (double)v * scale + 6755399441055744.0;  // 1.5 * 2^52
    return __double_as_longlong(t) - 0x4338000000000000ll;
}
__device__ __forceinline__ float bwd_from_fixed(long long t, int S) {
    return (float)ldexp((double)t, -S);
}

// Block reduction for a backward tile: the box (lx, hx, ly, hy) of the
// corner pixels and the largest |g| as float bits (non-negative floats order
// like their bit patterns).  Ends with a barrier.
__device__ __forceinline__ void bwd_block_reduce(int& lx, int& hx, int& ly, int& hy, int& mb, int* box) {
    const int tid = threadIdx.x;
    lx = wave_min(lx); hx = wave_max(hx); ly = wave_min(ly); hy = wave_max(hy); mb = wave_max(mb);
    const int wv = tid >> 6;
    __syncthreads();  // earlier readers of box are done
    if ((tid & 63) == 0) {
        box[5 * wv] = lx; box[5 * wv + 1] = hx; box[5 * wv + 2] = ly; box[5 * wv + 3] = hy; box[5 * wv + 4] = mb;
    }
    __syncthreads();
    lx = box[0]; hx = box[1]; ly = box[2]; hy = box[3]; mb = box[4];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        lx = min(lx, box[5 * w]); hx = max(hx, box[5 * w + 1]);
        ly = min(ly, box[5 * w + 2]); hy = max(hy, box[5 * w + 3]); mb = max(mb, box[5 * w + 4]);
    }
}

// One 16 x 16 tile of queries.  The tile's scatter into dXii is summed in an
// LDS window covering every corner its queries touch (fixed point, above) and
// then added to global memory once per window entry, in row order; a tile
// whose window exceeds kBwdLdsPx, or whose largest |g| is zero, subnormal or
// not finite, adds each corner to global memory directly.  All 256 lanes of
// the block call this; it ends without a barrier, so a caller that reuses acc
// for another tile synchronises first.
__device__ __forceinline__ void bwd_tile(const BwdEdgeArgs& B, int tile, unsigned long long* acc, int* box) {
    const int H = B.H, W = B.W;
    const int tid = threadIdx.x;
    // The whole accumulator is cleared up front, overlapped with the query
    // reads; the barriers of the block reduction order it before the atomics.
    for (int i = tid; i < kBwdAccWords / 2; i += 256)
        reinterpret_cast<float4*>(acc)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int x = (tile % B.tiles_x) * 16 + (tid & 15), y = (tile / B.tiles_x) * 16 + (tid >> 4);
    const bool inside = x < W && y < H;
    const long n = (long)y * W + x;
    const bool has_gx = B.grad_xhat != nullptr;
    long cm[4] = {-1, -1, -1, -1};
    float3 gc[4];
    int lx = INT_MAX, hx = INT_MIN, ly = INT_MAX, hy = INT_MIN, mb = 0;
    int cx0 = 0, cy0 = 0;  // cell of p*: corner c is (cx0 + (c & 1), cy0 + (c >> 1))
    if (inside) {
        BwdQueryIn in;
        const bool valid = ld_global(B.valid, n) != 0;
        in.px = ld_global(B.p, 2 * n); in.py = ld_global(B.p, 2 * n + 1);
        in.gp0 = ld_global(B.grad_p, 2 * n); in.gp1 = ld_global(B.grad_p, 2 * n + 1);
        in.gx = has_gx ? ld_global_point(B.grad_xhat, n) : f3(0.f, 0.f, 0.f);
        in.xq = ld_global_point(B.Xji, n);
        float3 dq = f3(0.f, 0.f, 0.f);
        if (valid) {
            dq = bwd_query(H, W, B.Xii, has_gx, in, cm, gc, cx0, cy0);
            lx = cx0; hx = cx0 + 1; ly = cy0; hy = cy0 + 1;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (cm[c] < 0) continue;
                const uint32_t m3 = max(max(__float_as_uint(fabsf(gc[c].x)), __float_as_uint(fabsf(gc[c].y))),
                                        __float_as_uint(fabsf(gc[c].z)));
                mb = max(mb, (int)m3);
            }
        }
        __attribute__((address_space(1))) float* dXji = (__attribute__((address_space(1))) float*)B.dXji;
        dXji[3 * n] = dq.x; dXji[3 * n + 1] = dq.y; dXji[3 * n + 2] = dq.z;
    }
    bwd_block_reduce(lx, hx, ly, hy, mb, box);
    const int bw = hx - lx + 1, bh = hy - ly + 1;
    const bool any = hx >= lx;
    const int ge = mb >> 23;  // biased exponent of the largest |g| (255: inf or NaN)
    float* __restrict__ dXii = B.dXii;
    if (any && ge > 0 && ge < 255 && bw * bh <= kBwdLdsPx) {
        const int S = 49 - (ge - 127);
        const double scale = ldexp(1.0, S);
        // Planar accumulator: component k of window pixel j at acc[k * kBwdPlane + j].
        const int np = bw * bh;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (cm[c] < 0) continue;
            const int cy = cy0 + (c >> 1), cx = cx0 + (c & 1);
            unsigned long long* a = acc + (cy - ly) * bw + (cx - lx);
            atomicAdd(a, (unsigned long long)bwd_to_fixed(gc[c].x, scale));
            atomicAdd(a + kBwdPlane, (unsigned long long)bwd_to_fixed(gc[c].y, scale));
            atomicAdd(a + 2 * kBwdPlane, (unsigned long long)bwd_to_fixed(gc[c].z, scale));
        }
        __syncthreads();
        // Window entry i (row-major over pixels, then components) to dXii.
        const SmallDiv div_row(3 * bw);
        for (int i = tid; i < 3 * np; i += 256) {
            const int row = div_row(i), col = i - row * 3 * bw;
            const int px = col / 3, k = col - 3 * px;
            const long long t = (long long)acc[k * kBwdPlane + row * bw + px];
            if (t == 0) continue;
            add_global(dXii + 3 * ((long)(ly + row) * W + lx) + col, bwd_from_fixed(t, S));
        }
    } else {
        if (any && tid == 0) count_path(kPathBwdDirect);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (cm[c] < 0) continue;
            add_global(dXii + 3 * cm[c] + 0, gc[c].x);
            add_global(dXii + 3 * cm[c] + 1, gc[c].y);
            add_global(dXii + 3 * cm[c] + 2, gc[c].z);
        }
    }
}

__global__ void __launch_bounds__(256) bwd_kernel(BwdEdgeArgs B) {
    __shared__ __align__(16) unsigned long long acc[kBwdAccWords];
    __shared__ int box[5 * 4];
    bwd_tile(B, blockIdx.x, acc, box);
}

// Zeroes dXii of every edge of a batched backward (blockIdx.y = edge, grid-
// stride over blockIdx.x).
__global__ void __launch_bounds__(256) batched_bwd_zero_kernel(const BwdEdgeArgs* __restrict__ E) {
    const BwdEdgeArgs& B = E[blockIdx.y];
    float* __restrict__ a = B.dXii;
    const long count = 3L * B.H * B.W;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    const long head = min(count, (long)(((16u - ((uint32_t)(uintptr_t)a & 15u)) & 15u) >> 2));
    if (i < head) a[i] = 0.f;
    float4* __restrict__ b = reinterpret_cast<float4*>(a + head);
    const long nb = (count - head) >> 2;
    for (long j = i; j < nb; j += stride) store_nt(b + j, make_float4(0.f, 0.f, 0.f, 0.f));
    const long t = head + (nb << 2) + i;
    if (t < count && i < 4) a[t] = 0.f;
}

// Edge of a global backward tile id: the last edge whose tile_begin <= tile.
__device__ __forceinline__ int find_bwd_edge(const BwdEdgeArgs* __restrict__ E, int n_edges, int tile) {
    int lo = 0, hi = n_edges - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (E[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Backward over every edge with a fixed assignment of tiles to workgroups (the
// tiles cost about the same, so no queue: a single global counter serialises
// its atomics at one address, which took most of the launch).  The dispatcher
// hands workgroups to the XCDs round robin, so workgroup b runs on XCD b mod
// bands; each XCD takes one contiguous band of tiles, and neighbouring tiles,
// whose corner windows overlap, share that XCD's L2.  dXii of every edge was
// zeroed by the previous launch.
__global__ void __launch_bounds__(256) batched_bwd_kernel(const BwdEdgeArgs* __restrict__ E, int n_edges,
                                                          int total_tiles) {
    __shared__ __align__(16) unsigned long long acc[kBwdAccWords];
    __shared__ int box[5 * 4];
    const int g = (int)gridDim.x, b = (int)blockIdx.x;
    const int bands = min(kXcds, g);
    const int x = b % bands, l = b / bands;
    const int per = (g - x + bands - 1) / bands;  // workgroups of this band
    const int band = (total_tiles + bands - 1) / bands;
    const int lo = x * band, hi = min(lo + band, total_tiles);
    for (int tile = lo + l; tile < hi; tile += per) {
        const int e = find_bwd_edge(E, n_edges, tile);
        const BwdEdgeArgs B = E[e];
        bwd_tile(B, tile - B.tile_begin, acc, box);
        __syncthreads();  // the tile's reads of acc are done before the next clears it
    }
}

// ---------------------------------------------------------------- match statistics

// Copies `words` 32-bit words from pinned host memory (read over the bus by
// the kernel itself) to device memory: for the small edge tables a kernel in
// the stream starts sooner than a DMA copy.
__global__ void __launch_bounds__(256) host_copy_kernel(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                        long words) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ a, long count) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    for (; i < count; i += stride) a[i] = 0u;
}

// counts[0] += valid queries, counts[1] += reference pixels whose bit this
// lane set first; one pair of atomics per wave.
__global__ void __launch_bounds__(256) stats_kernel(const int32_t* __restrict__ idx, const uint8_t* __restrict__ valid,
                                                    long N, long M, uint32_t* __restrict__ bitmap,
                                                    int32_t* __restrict__ counts) {
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    bool v = false, first = false;
    if (n < N && valid[n]) {
        int32_t m = idx[n];
        if (m >= 0 && m < M) {
            v = true;
            uint32_t bit = 1u << (m & 31);
            uint32_t old = atomicOr(bitmap + (m >> 5), bit);
            first = (old & bit) == 0u;
        }
    }
    unsigned long long bv = __ballot(v), bf = __ballot(first);
    if ((threadIdx.x & 63) == 0) {
        if (bv) atomicAdd(counts, (int32_t)__popcll(bv));
        if (bf) atomicAdd(counts + 1, (int32_t)__popcll(bf));
    }
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(long count, int per) { return (unsigned)((count + per - 1) / per); }

hipError_t launch_prep(const float* Xii, float4* rays, int H, int W, hipStream_t s) {
    timer_begin("prep", s);
    prep_kernel<<<(unsigned)prep_tiles(H, W), 256, 0, s>>>(Xii, rays, H, W);
    timer_end(s);
    return hipGetLastError();
}

template <int TX, int TY>
static void launch_fwd_tile(const EdgeArgs& A, bool desc_regs, int mode, bool remap, hipStream_t s) {
    const int tiles = ((A.W + TX - 1) / TX) * ((A.H + TY - 1) / TY);
    const int grid = remap ? ((tiles + kXcds - 1) / kXcds) * kXcds : tiles;
    const int rm = remap ? 1 : 0;
    if (mode == 2 && desc_regs && A.levels > 1)
        fwd_f16_kernel<TX, TY, true><<<grid, TX * TY, 0, s>>>(A, rm);
    else if (mode == 2 && desc_regs)
        fwd_f16_kernel<TX, TY, false><<<grid, TX * TY, 0, s>>>(A, rm);
    else if (mode == 1 && desc_regs)
        fwd_lds_kernel<TX, TY><<<grid, TX * TY, 0, s>>>(A, rm);
    else if (desc_regs)
        fwd_kernel<TX, TY, 24><<<grid, TX * TY, 0, s>>>(A, rm);
    else
        fwd_kernel<TX, TY, 0><<<grid, TX * TY, 0, s>>>(A, rm);
}

void tile_shape(int tile_config, int* tx, int* ty) {
    switch (tile_config) {
        case 1: case 3: case 5: *tx = 16; *ty = 16; return;
        case 2: *tx = 64; *ty = 4; return;
        case 6: *tx = 8; *ty = 8; return;
        default: *tx = 32; *ty = 8; return;
    }
}

bool tile_uses_lds(int tile_config) { return tile_config >= 3; }

hipError_t launch_fwd(const EdgeArgs& A, int tile_config, bool desc_regs, bool xcd_remap, hipStream_t s) {
    timer_begin("fwd", s);
    switch (tile_config) {
        case 1: launch_fwd_tile<16, 16>(A, desc_regs, 0, xcd_remap, s); break;
        case 2: launch_fwd_tile<64, 4>(A, desc_regs, 0, xcd_remap, s); break;
        case 3: launch_fwd_tile<16, 16>(A, desc_regs, 1, xcd_remap, s); break;
        case 4: launch_fwd_tile<32, 8>(A, desc_regs, 1, xcd_remap, s); break;
        case 5: launch_fwd_tile<16, 16>(A, desc_regs, 2, xcd_remap, s); break;
        case 6: launch_fwd_tile<8, 8>(A, desc_regs, 2, xcd_remap, s); break;
        default: launch_fwd_tile<32, 8>(A, desc_regs, 0, xcd_remap, s); break;
    }
    timer_end(s);
    return hipGetLastError();
}

template <int TX, int TY, int MARGIN, int UNROLL>
static void launch_batched_f16(const EdgeArgs* table, int n_edges, int total_tiles, int32_t* counter, int grid,
                               hipStream_t s) {
    batched_fwd_kernel<TX, TY, 24, 2, MARGIN, UNROLL><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles, counter);
}

template <int TX, int TY>
static void launch_batched_tile(const EdgeArgs* table, int n_edges, int total_tiles, int32_t* counter, int grid,
                                bool desc_regs, int mode, int margin, int unroll, int levels, hipStream_t s) {
    if constexpr (TX == 16 && TY == 16) {
        if (mode == 2 && desc_regs && levels > 1) {
            batched_fwd_kernel<TX, TY, 24, 2, kRayMargin, 1, true><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles,
                                                                                        counter);
            return;
        }
        if (mode == 2 && desc_regs) {
            const int v = 2 * (margin - 1) + (unroll - 1);
            switch (v) {
                case 0: launch_batched_f16<TX, TY, 1, 1>(table, n_edges, total_tiles, counter, grid, s); break;
                case 1: launch_batched_f16<TX, TY, 1, 2>(table, n_edges, total_tiles, counter, grid, s); break;
                case 3: launch_batched_f16<TX, TY, 2, 2>(table, n_edges, total_tiles, counter, grid, s); break;
                case 4: launch_batched_f16<TX, TY, 3, 1>(table, n_edges, total_tiles, counter, grid, s); break;
                case 5: launch_batched_f16<TX, TY, 3, 2>(table, n_edges, total_tiles, counter, grid, s); break;
                default: launch_batched_f16<TX, TY, 2, 1>(table, n_edges, total_tiles, counter, grid, s); break;
            }
            return;
        }
    } else {
        if (mode == 2 && desc_regs) {
            if (levels > 1)
                batched_fwd_kernel<TX, TY, 24, 2, kRayMargin, 1, true><<<grid, TX * TY, 0, s>>>(table, n_edges,
                                                                                            total_tiles, counter);
            else
                batched_fwd_kernel<TX, TY, 24, 2><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles, counter);
            return;
        }
    }
    if (mode == 1 && desc_regs)
        batched_fwd_kernel<TX, TY, 24, 1><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles, counter);
    else if (desc_regs)
        batched_fwd_kernel<TX, TY, 24, 0><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles, counter);
    else
        batched_fwd_kernel<TX, TY, 0, 0><<<grid, TX * TY, 0, s>>>(table, n_edges, total_tiles, counter);
}

hipError_t launch_batched(const EdgeArgs* table, const int32_t* prep_begin, int n_edges, int total_prep_blocks,
                          int total_tiles, int32_t* counter, int tile_config, int grid, int margin, int unroll,
                          int levels, bool desc_regs, hipStream_t s) {
    timer_begin("batched_prep", s);
    batched_prep_kernel<<<total_prep_blocks, 256, 0, s>>>(table, prep_begin, n_edges, counter);
    timer_end(s);
    timer_begin("batched_fwd", s);
    switch (tile_config) {
        case 1: launch_batched_tile<16, 16>(table, n_edges, total_tiles, counter, grid, desc_regs, 0, margin, unroll, levels, s); break;
        case 2: launch_batched_tile<64, 4>(table, n_edges, total_tiles, counter, grid, desc_regs, 0, margin, unroll, levels, s); break;
        case 3: launch_batched_tile<16, 16>(table, n_edges, total_tiles, counter, grid, desc_regs, 1, margin, unroll, levels, s); break;
        case 4: launch_batched_tile<32, 8>(table, n_edges, total_tiles, counter, grid, desc_regs, 1, margin, unroll, levels, s); break;
        case 5: launch_batched_tile<16, 16>(table, n_edges, total_tiles, counter, grid, desc_regs, 2, margin, unroll, levels, s); break;
        case 6: launch_batched_tile<8, 8>(table, n_edges, total_tiles, counter, grid, desc_regs, 2, margin, unroll, levels, s); break;
        default: launch_batched_tile<32, 8>(table, n_edges, total_tiles, counter, grid, desc_regs, 0, margin, unroll, levels, s); break;
    }
    timer_end(s);
    return hipGetLastError();
}

hipError_t launch_host_copy(void* dst, const void* pinned_src, size_t bytes, hipStream_t s) {
    const long words = (long)(bytes / 4);
    host_copy_kernel<<<min(blocks_for(words, 256), 64u), 256, 0, s>>>(static_cast<uint32_t*>(dst),
                                                                      static_cast<const uint32_t*>(pinned_src), words);
    return hipGetLastError();
}

hipError_t launch_stats(const int32_t* idx, const uint8_t* valid, int H, int W, uint32_t* bitmap, int32_t* counts,
                        hipStream_t s) {
    long N = (long)H * W;
    long words = (N + 31) / 32;
    timer_begin("stats_fill", s);
    fill_u32_kernel<<<min(blocks_for(words + 2, 256), 1024u), 256, 0, s>>>(bitmap, words);
    fill_u32_kernel<<<1, 64, 0, s>>>(reinterpret_cast<uint32_t*>(counts), 2);
    timer_end(s);
    timer_begin("stats", s);
    stats_kernel<<<blocks_for(N, 256), 256, 0, s>>>(idx, valid, N, N, bitmap, counts);
    timer_end(s);
    return hipGetLastError();
}

hipError_t read_path_counters(int64_t* out, bool reset) {
    hipError_t e = hipDeviceSynchronize();
    unsigned long long v[kNumPathCounters];
    if (e == hipSuccess) e = hipMemcpyFromSymbol(v, HIP_SYMBOL(g_path_counts), sizeof v, 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kNumPathCounters; ++k) out[k] = (int64_t)v[k];
    if (reset) {
        for (int k = 0; k < kNumPathCounters; ++k) v[k] = 0ull;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_path_counts), v, sizeof v, 0, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    return e;
}

hipError_t launch_bwd(const BwdEdgeArgs& B, hipStream_t s) {
    long N = (long)B.H * B.W;
    timer_begin("fill", s);
    fill_zero_kernel<<<min(blocks_for(3 * N / 4 + 1, 256), 4096u), 256, 0, s>>>(B.dXii, 3 * N);
    timer_end(s);
    timer_begin("bwd", s);
    bwd_kernel<<<B.tiles_x * B.tiles_y, 256, 0, s>>>(B);
    timer_end(s);
    return hipGetLastError();
}

hipError_t launch_bwd_batched(const BwdEdgeArgs* table, int n_edges, long max_pixels, int total_tiles, int grid,
                              bool zero, hipStream_t s) {
    if (zero) {
        timer_begin("batched_bwd_zero", s);
        const unsigned zx = min(blocks_for(3 * max_pixels / 4 + 1, 256), 1024u);
        batched_bwd_zero_kernel<<<dim3(zx, (unsigned)n_edges), 256, 0, s>>>(table);
        timer_end(s);
    }
    timer_begin("batched_bwd", s);
    batched_bwd_kernel<<<grid, 256, 0, s>>>(table, n_edges, total_tiles);
    timer_end(s);
    return hipGetLastError();
}

}  // namespace m3s
