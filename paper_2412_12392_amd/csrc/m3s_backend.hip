// gfx950 kernels of the backend optimisation (MASt3R-SLAM, Sec. 3.5).
//
// Gauss-Newton over the world poses T_WC of N keyframes on the global ray
// objective (Eq. backend_ray) plus the small-weight distance term, summed over
// every edge (i, j) and every valid match (n of keyframe j, m = idx[n] of
// keyframe i) with confidence q = sqrt(Q_i[m] Q_j[n]) > q_min.  The residuals
// of an edge depend on the relative pose T_ij = T_WC[i]^-1 T_WC[j] only, and
// the world-pose Jacobians are -J Ad(T_WC[i]^-1) and J Ad(T_WC[i]^-1) (Supp. A,
// relative to global pose), so with A = Ad(T_WC[i]^-1) an edge contributes
//   H_ii += A^T H_e A,  H_jj += A^T H_e A,  H_ij = H_ji^T -= A^T H_e A,
//   g_i  -= A^T g_e,    g_j  += A^T g_e
// where (H_e, g_e) are the edge's 7x7 normal equations w.r.t. a left
// perturbation of T_ij.  Per iteration:
//
//   accum   grid (blocks, edges): every lane sums the relative normal
//           equations of its matches in fp32 (the tracking residuals with
//           x = T_ij X_j[n] transformed and X_i[m] measured); one partial per
//           workgroup.
//   edge    one workgroup per edge: the edge's partials summed in fp64 in a
//           fixed order; A^T H_e A and A^T g_e.
//   assemble one workgroup per block row of the reduced 7(N-1) system
//           (keyframe 0 holds the gauge): the edges' blocks summed in LDS in
//           edge order, one writer per entry, rows written out whole.
//   solve   one workgroup: the block-sparse Cholesky of the system in
//           keyframe order over its fill pattern (found once per call), in
//           LDS, the forward substitution folded into the factorization;
//           when the fill exceeds LDS, the dense blocked right-looking
//           Cholesky in fp64 with 32 x 32 tiles instead (the diagonal tile
//           factored one column group per barrier, the panel kept in LDS, the
//           backward substitution blocked);
//           T_WC[k] <- Exp(tau_k) o T_WC[k] (Eq. 1).  A system that is not positive definite, or a step norm
//           below step_tol, ends the loop: later launches of the call return
//           at once.
//
// Kernel boundaries order every hand-off, so no workgroup needs a
// device-scope fence.  A final accumulation at the last poses gives the cost
// and match count.  Launches are stream-ordered with no host synchronisation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m3s.h"
#include "m3s_internal.h"
#include "m3s_sim3.h"

namespace m3s {

namespace {

constexpr int kThreads = 256;
constexpr int kSolveThreads = 512;
constexpr int kVals = kPoseVals;
constexpr int kStride = 40;         // floats per block partial, doubles per edge system
constexpr int kMaxDim = 7 * (M3S_MAX_KEYFRAMES - 1);  // largest reduced system
constexpr int kPatWords = (M3S_MAX_KEYFRAMES + 31) / 32;  // bit words per block row of the pattern

struct BackendArgs {
    int N, HW, E, blocks_per_edge;
    int n, np;                // reduced system size 7(N-1) and its padding to whole tiles
    const float* Xc;          // [N*HW*3]
    const float* Q;           // [N*HW]
    const int32_t* edges;     // [E*2] (i, j)
    const int32_t* idx;       // [E*HW]
    const uint8_t* valid;     // [E*HW]
    double q_min;
    float q_minf;
    RobustWeights rw;
    double step_tol;
    double* T64;              // [N*12] world poses
    float* Trel;              // [E*12] T_ij = T_WC[i]^-1 T_WC[j] per edge at the current poses (zero out of range)
    double* edge_sys;         // [E*kStride] fp64 relative normal equations per edge
    double* edge_blk;         // [E*kBlk] A^T H_e A (49) and A^T g_e (7) per edge
    float* partials;          // [E*blocks_per_edge*kStride]
    int32_t* state;           // [0] done flag, [1] applied steps, [2] the factor's fill exceeds the sparse solve
    double* stat;             // [0] last step norm
    double* M;                // [np*np] reduced Hessian, factored in place (lower triangle)
    double* rhs;              // [np]
    double* dinv;             // [nt*kTile*kTile] inverses of the diagonal tiles
    uint32_t* pat;            // [(N-1)*kPatWords] block pattern of the factor L (lower, after fill), bit j of row i
    int32_t* row_start;       // [N] first slot of each block row of L in row-major block order; [N-1] = blocks
    float* T_out;             // [N*12]
    float* info;              // [4] or null
};

constexpr int kBlk = 56;      // 49 + 7 doubles per edge
constexpr int kMatchesPerLane = 16;  // amortises the workgroup reduction of the 37 sums
constexpr int kTile = 32;     // tile of the blocked Cholesky
constexpr int kPanelRows = 416;  // panel rows kept in LDS (larger systems read the panel from memory)
constexpr int kStageRows = 64;   // raw panel rows staged per step of the panel product
constexpr int kPanelStride = kTile + 1;  // odd stride in doubles: rows of a wave fall in different banks

__global__ void __launch_bounds__(256) backend_init_kernel(const float* __restrict__ T_in, double* __restrict__ T64,
                                                           int N, int32_t* __restrict__ state,
                                                           double* __restrict__ stat) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 12 * N) T64[t] = (double)T_in[t];
    if (t < 3) state[t] = 0;
    if (t < 2) stat[t] = 0.0;
}

__device__ __forceinline__ bool edge_in_range(int ei, int ej, int N) {
    return ei >= 0 && ei < N && ej >= 0 && ej < N;
}

// T_ij of edge e in fp32 from the fp64 world poses (zero for an edge out of range).
__device__ __forceinline__ void write_relative_pose(const BackendArgs& A, int e) {
    const int ei = A.edges[2 * e], ej = A.edges[2 * e + 1];
    double Ti[12], Tij[12];
    if (edge_in_range(ei, ej, A.N)) {
        sim3_inverse(A.T64 + 12 * ei, Ti);
        sim3_mul(Ti, A.T64 + 12 * ej, Tij);
    } else {
        for (int k = 0; k < 12; ++k) Tij[k] = 0.0;
    }
    for (int k = 0; k < 12; ++k) A.Trel[12 * e + k] = (float)Tij[k];
}

// Relative poses at the initial world poses, one thread per edge.
__global__ void __launch_bounds__(256) backend_relpose_kernel(BackendArgs A) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < A.E) write_relative_pose(A, e);
}

// final: 0 = an iteration's accumulation (skipped once the loop has ended), 1 = the final one.
__global__ void __launch_bounds__(kThreads) backend_accum_kernel(BackendArgs A, int final_pass) {
    __shared__ float red[kThreads / 64][kVals];
    if (!final_pass && A.state[0]) return;
    const int e = blockIdx.y;
    const int ei = A.edges[2 * e], ej = A.edges[2 * e + 1];
    const bool edge_ok = edge_in_range(ei, ej, A.N);
    float T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = A.Trel[12 * e + k];
    float acc[kVals];
#pragma unroll
    for (int k = 0; k < kVals; ++k) acc[k] = 0.f;

    const long ebase = (long)e * A.HW;
    const float* Xi = A.Xc + (long)(edge_ok ? ei : 0) * A.HW * 3;
    const float* Xj = A.Xc + (long)(edge_ok ? ej : 0) * A.HW * 3;
    const float* Qi = A.Q + (long)(edge_ok ? ei : 0) * A.HW;
    const float* Qj = A.Q + (long)(edge_ok ? ej : 0) * A.HW;
    // Workgroups are dealt to the 8 XCDs round-robin (b % 8 with the edge's
    // workgroups consecutive); chunk c(b) gives XCD j the j-th contiguous
    // eighth of the chunks, so each XCD's L2 sees one slice of every keyframe
    // and the edges that share a keyframe reuse it there.
    const int bpe = A.blocks_per_edge;
    const int chunk = (bpe % 8 == 0) ? (int)(blockIdx.x % 8) * (bpe / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const int stride = bpe * kThreads;
    // kBatch consecutive matches of the lane (same order as one at a time)
    // have their reads issued together before the arithmetic.
    constexpr int kBatch = 4;
    for (int n0 = edge_ok ? chunk * kThreads + threadIdx.x : A.HW; n0 < A.HW; n0 += kBatch * stride) {
        int nn[kBatch], mm[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            nn[u] = n0 + u * stride;
            ok[u] = nn[u] < A.HW && A.valid[ebase + nn[u]];
            mm[u] = ok[u] ? A.idx[ebase + nn[u]] : 0;
            ok[u] = ok[u] && mm[u] >= 0 && mm[u] < A.HW;
        }
        float qi[kBatch], qj[kBatch], xi[kBatch][3], xj[kBatch][3];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int m = ok[u] ? mm[u] : 0, n = ok[u] ? nn[u] : 0;
            qi[u] = Qi[m]; qj[u] = Qj[n];
#pragma unroll
            for (int j = 0; j < 3; ++j) { xi[u][j] = Xi[3 * m + j]; xj[u][j] = Xj[3 * n + j]; }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            float q;
            if (ok[u] && confidence_gate(qi[u], qj[u], A.q_min, A.q_minf, q))
                accumulate_match(T, xj[u][0], xj[u][1], xj[u][2], xi[u][0], xi[u][1], xi[u][2], q, A.rw, acc);
        }
    }

#pragma unroll
    for (int k = 0; k < kVals; ++k) acc[k] = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < kVals; ++k) red[threadIdx.x >> 6][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < kVals) {
        float v = 0.f;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
        A.partials[((size_t)e * A.blocks_per_edge + blockIdx.x) * kStride + threadIdx.x] = v;
    }
}

// One workgroup per edge: fixed-order fp64 sum of the edge's partials; then
// (iterations only) A = Ad(T_WC[i]^-1), A^T H_e A and A^T g_e.
__global__ void __launch_bounds__(kThreads) backend_edge_kernel(BackendArgs A, int final_pass) {
    __shared__ double sys[kStride];
    __shared__ double part[kThreads / kVals * kVals];
    __shared__ double Ad[49];
    if (!final_pass && A.state[0]) return;
    const int e = blockIdx.x;
    sum_partials<kThreads>(A.partials + (size_t)e * A.blocks_per_edge * kStride, A.blocks_per_edge, kStride, part, sys);
    if (threadIdx.x < kVals) A.edge_sys[(size_t)e * kStride + threadIdx.x] = sys[threadIdx.x];
    if (final_pass) return;
    const int ei = A.edges[2 * e], ej = A.edges[2 * e + 1];
    if (!edge_in_range(ei, ej, A.N)) return;
    if (threadIdx.x == 0) {
        double Ti[12];
        sim3_inverse(A.T64 + 12 * ei, Ti);
        sim3_adjoint(Ti, Ad);
    }
    __syncthreads();
    double* out = A.edge_blk + (size_t)e * kBlk;
    if (threadIdx.x < 49) {
        const int a = threadIdx.x / 7, b = threadIdx.x % 7;
        double s = 0.0;
        for (int k = 0; k < 7; ++k) {
            double hk = 0.0;
            for (int l = 0; l < 7; ++l) hk += sys[upper_index(k < l ? k : l, k < l ? l : k)] * Ad[7 * l + b];
            s += Ad[7 * k + a] * hk;
        }
        out[threadIdx.x] = s;
    } else if (threadIdx.x >= 64 && threadIdx.x < 71) {
        const int a = threadIdx.x - 64;
        double s = 0.0;
        for (int k = 0; k < 7; ++k) s += Ad[7 * k + a] * sys[28 + k];
        out[49 + a] = s;
    }
}

// Assembly of the reduced system: one workgroup per block row (keyframe
// p = blockIdx.x + 1, rows 7(p-1) .. 7(p-1)+6) and one for the padding rows.
// The row block is summed in LDS from the edges' blocks in edge order (thread
// (a, b) owns the entries at offset (a, b) of the diagonal block, thread
// 64 + (a, b) those of the off-diagonal blocks, so every entry has one writer,
// which visits the edges in order) and written out whole, zeros included,
// with its right-hand side -g.
constexpr int kAsmThreads = 128;
constexpr int kMaxNp = (kMaxDim + kTile - 1) / kTile * kTile;

__global__ void __launch_bounds__(kAsmThreads) backend_assemble_kernel(BackendArgs A) {
    __shared__ double rows[7 * kMaxNp];
    __shared__ double rr[7];
    if (A.state[0]) return;
    const int np = A.np, n = A.n, tid = threadIdx.x;
    if ((int)blockIdx.x == A.N - 1) {
        for (int r = n; r < np; ++r)
            for (int c = tid; c < np; c += kAsmThreads) A.M[(long)r * np + c] = r == c ? 1.0 : 0.0;
        for (int r = n + tid; r < np; r += kAsmThreads) A.rhs[r] = 0.0;
        return;
    }
    for (int i = tid; i < 7 * np; i += kAsmThreads) rows[i] = 0.0;
    if (tid < 7) rr[tid] = 0.0;
    __syncthreads();
    const int P = (int)blockIdx.x + 1, I = 7 * (P - 1);
    const int a = (tid & 63) / 7, b = (tid & 63) % 7;
    for (int e = 0; e < A.E; ++e) {
        const int ei = A.edges[2 * e], ej = A.edges[2 * e + 1];
        // A self edge has T_ij = I whatever the poses: its blocks cancel.
        if (!edge_in_range(ei, ej, A.N) || ei == ej) continue;
        const bool own_i = ei == P;
        if (!own_i && ej != P) continue;
        const double* blk = A.edge_blk + (size_t)e * kBlk;
        const int other = own_i ? ej : ei;
        if (tid < 49) {
            // H_ii += A^T H_e A (own_i), H_jj += A^T H_e A (own_j)
            rows[a * np + I + b] += blk[7 * a + b];
        } else if (tid >= 64 && tid < 64 + 49) {
            // H_ij -= A^T H_e A, H_ji -= (A^T H_e A)^T; keyframe 0 holds the gauge
            if (other > 0) rows[a * np + 7 * (other - 1) + b] -= own_i ? blk[7 * a + b] : blk[7 * b + a];
        } else if (tid >= 49 && tid < 56) {
            // right-hand side -g: g_i -= A^T g_e, g_j += A^T g_e
            const int o = tid - 49;
            rr[o] += own_i ? blk[49 + o] : -blk[49 + o];
        }
    }
    __syncthreads();
    for (int i = tid; i < 7 * np; i += kAsmThreads) {
        const int r = i / np, c = i - r * np;
        A.M[(long)(I + r) * np + c] = rows[i];
    }
    if (tid < 7) A.rhs[I + tid] = rr[tid];
}

// Tile (ti, tj) of M as kTile x kTile, row-major with leading dimension np.
__device__ __forceinline__ double* tile_ptr(const BackendArgs& A, int ti, int tj) {
    return A.M + (long)ti * kTile * A.np + (long)tj * kTile;
}

// Trailing update of one 32 x 32 tile (ti, tj), tj <= ti, of the lower
// triangle below tile column k: M[R][C] -= L[R] . L[C], a 4 x 4 block per lane
// of one wave.  P points at the panel rows (stride ps doubles): LDS or M.  Tile
// (0, 0) is the next diagonal tile: its lower triangle goes to dl (the LDS tile
// the next factor reads, stride kTile + 1) instead of M.
template <typename PanelPtr>
__device__ __forceinline__ void trailing_tile(const BackendArgs& A, PanelPtr P, int ps, int R0, int ti, int tj,
                                              int lane, double* dl) {
    const int np = A.np;
    const int r0 = (lane >> 3) * 4, c0 = (lane & 7) * 4;
    const int ra = ti * kTile + r0, ca = tj * kTile + c0;
    // The target entries are read first so their latency overlaps the product.
    double cur[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) cur[u][v] = A.M[(long)(R0 + ra + u) * np + R0 + ca + v];
    double acc[4][4] = {};
    for (int t = 0; t < kTile; ++t) {
        double va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            va[u] = P[(long)(ra + u) * ps + t];
            vb[u] = P[(long)(ca + u) * ps + t];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += va[u] * vb[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (ti != tj || c0 + v <= r0 + u) {
                const double val = cur[u][v] - acc[u][v];
                if (ti == 0 && tj == 0) dl[(r0 + u) * (kTile + 1) + c0 + v] = val;
                else A.M[(long)(R0 + ra + u) * np + R0 + ca + v] = val;
            }
}

// The end of a solve: pose updates T_WC[k] <- Exp(tau_k) o T_WC[k] for
// keyframes 1..N-1 from the solution x (LDS), the relative pose of every edge
// at the new poses (for the next accumulation), and the step norm, which ends
// the loop below step_tol.  All NT lanes of the workgroup call this.
template <int NT>
__device__ __forceinline__ void apply_step(const BackendArgs& A, const double* x, double* red) {
    const int tid = threadIdx.x;
    for (int k = 1 + tid; k < A.N; k += NT) {
        double E[12], Tn[12];
        sim3_exp(x + 7 * (k - 1), E);
        sim3_mul(E, A.T64 + 12 * k, Tn);
        for (int j = 0; j < 12; ++j) A.T64[12 * k + j] = Tn[j];
    }
    __syncthreads();
    for (int e = tid; e < A.E; e += NT) write_relative_pose(A, e);
    double sq = 0.0;
    for (int k = tid; k < A.n; k += NT) sq += x[k] * x[k];
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        const double step = sqrt(t);
        A.stat[0] = step;
        A.state[1] += 1;
        if (step < A.step_tol) A.state[0] = 1;
    }
}

// One workgroup: factor the assembled reduced system (blocked Cholesky),
// solve and update the poses.  Runs when the block-sparse factor does not fit
// (state[2]); otherwise backend_sparse_solve_kernel has solved the system.
__global__ void __launch_bounds__(kSolveThreads) backend_solve_kernel(BackendArgs A) {
    __shared__ double D[kTile][kTile + 1];        // diagonal tile being factored
    __shared__ double Dinv[kTile][kTile + 1];     // its inverse
    __shared__ double V[kTile][kTile + 1];        // the inverse's rows before scaling
    __shared__ double panel[kPanelRows * kPanelStride];  // the factored panel below it
    __shared__ double x[kMaxDim + kTile];          // right-hand side, then the solution
    __shared__ double red[kSolveThreads / 64];
    __shared__ double part[kTile];
    __shared__ double stage[kStageRows * kPanelStride];  // raw panel rows
    if (A.state[0] || !A.state[2]) return;
    const int tid = threadIdx.x;
    const int n = A.n, np = A.np, nt = np / kTile;

    for (int k = tid; k < np; k += kSolveThreads) x[k] = A.rhs[k];

    // Blocked right-looking Cholesky, lower triangle, kTile x kTile tiles.
    // Per tile column k: the diagonal tile is factored, its inverse
    // Dinv = L_kk^-1 is formed and kept for the substitutions, the panel below
    // becomes A_ik Dinv^T (a product, no sequential chain) and the trailing
    // lower triangle takes -= L_ik L_jk^T from the panel (in LDS when it fits).
    bool failed = false;  // the same in every thread: decided from LDS values read after a barrier
    for (int k = 0; k < nt; ++k) {
        double* Mk = tile_ptr(A, k, k);
        // Tile 0 comes from M; every later diagonal tile was left in D by the
        // previous trailing update (its lower triangle, the only part read).
        if (k == 0)
            for (int q = tid; q < kTile * kTile; q += kSolveThreads) D[q / kTile][q % kTile] = Mk[(long)(q / kTile) * np + q % kTile];
        for (int q = tid; q < kTile * kTile; q += kSolveThreads) V[q / kTile][q % kTile] = (q / kTile == q % kTile) ? 1.0 : 0.0;
        const int R0 = (k + 1) * kTile;
        const int m = np - R0;
        static_assert(kStageRows * kTile % kSolveThreads == 0, "whole raw values per thread");
        constexpr int kL = kStageRows * kTile / kSolveThreads;
        double raw[kL];
        auto read_stage = [&](int r0) {
#pragma unroll
            for (int j = 0; j < kL; ++j) {
                const int q = tid + j * kSolveThreads;
                const int rr = r0 + q / kTile, t = q % kTile;
                raw[j] = rr < m ? A.M[(long)(R0 + rr) * np + k * kTile + t] : 0.0;
            }
        };
        // The first panel stage's raw rows (below this tile, which the factor
        // does not write) are read before the factor, to arrive during it.
        if (m > 0) read_stage(0);
        __syncthreads();
        // Factor the tile with the whole workgroup, one barrier per step.  Per
        // column c, with d = D[c][c], the entries below take
        // D[r][q] -= D[r][c] D[q][c] / d and the rows of the running inverse
        // V[r][q] -= D[r][c] V[c][q] / d (r > c); the scaled outputs, column c
        // of L (to M) and row c of Dinv = L_kk^-1 = V[c] / sqrt(d), go to other
        // arrays.  A step takes a group of kC columns: every thread reads the
        // group's pivot block and its entries' values in the group's columns,
        // eliminates them through the group itself, and writes only entries
        // right of the group, rows of V below it, Dinv and M, so a step writes
        // nothing it reads.  Every thread forms the same pivots from the same
        // values read after a barrier, so the decision to stop is the same in
        // every thread.
        constexpr int kC = 4;  // columns per step
        static_assert(kTile % kC == 0, "whole column groups");
        for (int c = 0; c < kTile; c += kC) {
            // Two entries per thread.  Their operands (all inside the tile) are
            // read unconditionally together with the pivot block, so one LDS
            // round trip serves the step.
            static_assert(kTile * kTile % kSolveThreads == 0, "whole entries per thread");
            constexpr int kH = kTile * kTile / kSolveThreads;
            // Per entry: x = D[r][q] (entries right of the group) or V[r][q];
            // rc[l] = D[r][c+l]; y[l] = D[q][c+l] or V[c+l][q] to match x.
            double x[kH], rc[kH][kC], y[kH][kC];
#pragma unroll
            for (int h = 0; h < kH; ++h) {
                const int e2 = tid + h * kSolveThreads;
                const int r = e2 / kTile, q = e2 % kTile;
                const bool d_ent = q >= c + kC && q <= r;
                x[h] = d_ent ? D[r][q] : V[r][q];
#pragma unroll
                for (int l = 0; l < kC; ++l) {
                    rc[h][l] = D[r][c + l];
                    y[h][l] = d_ent ? D[q][c + l] : V[c + l][q];
                }
            }
            // The group's pivot block (lower triangle), eliminated by every thread.
            double B[kC][kC];
#pragma unroll
            for (int i = 0; i < kC; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j) B[i][j] = D[c + i][c + j];
            bool bad = false;
            double isv[kC], sdv[kC];
            double mk[kH], dv[kH];
#pragma unroll
            for (int h = 0; h < kH; ++h) mk[h] = dv[h] = 0.0;
#pragma unroll
            for (int j = 0; j < kC; ++j) {
                const double dj = B[j][j];
                bad = bad || !(dj > 0.0) || !isfinite(dj);
                // 1/sqrt(d): hardware estimate and two Newton steps.
                double is = __builtin_amdgcn_rsq(dj);
                is = is * fma(-0.5 * dj * is, is, 1.5);
                is = is * fma(-0.5 * dj * is, is, 1.5);
                const double idg = is * is;
                isv[j] = is;
                sdv[j] = dj * is;
#pragma unroll
                for (int i = j + 1; i < kC; ++i)
#pragma unroll
                    for (int l = j + 1; l <= i; ++l) B[i][l] -= B[i][j] * B[l][j] * idg;
#pragma unroll
                for (int h = 0; h < kH; ++h) {
                    const int e2 = tid + h * kSolveThreads;
                    const int r = e2 / kTile, q = e2 % kTile;
                    // Outputs of column c + j: L[r][c+j] and row c + j of Dinv.
                    if (q == c + j) mk[h] = rc[h][j] * is;
                    if (r == c + j) dv[h] = y[h][j] * is;
                    x[h] -= rc[h][j] * y[h][j] * idg;
#pragma unroll
                    for (int l = j + 1; l < kC; ++l) {
                        rc[h][l] -= rc[h][j] * B[l][j] * idg;
                        y[h][l] -= y[h][j] * B[l][j] * idg;
                    }
                }
            }
            if (bad) {
                failed = true;
                break;
            }
            // Each entry has at most one LDS output (D, V or a row of Dinv),
            // chosen by selects; the group's columns of L go to memory.
#pragma unroll
            for (int h = 0; h < kH; ++h) {
                const int e2 = tid + h * kSolveThreads;
                const int r = e2 / kTile, q = e2 % kTile;
                const bool d_upd = q >= c + kC && q <= r;
                const bool v_upd = r >= c + kC && q < c + kC;
                const bool i_row = r >= c && r < c + kC && q <= r;
                const double val = i_row ? dv[h] : x[h];
                double* dst = d_upd ? &D[r][q] : (v_upd ? &V[r][q] : &Dinv[r][q]);
                if (d_upd || v_upd || i_row) *dst = val;
                if (q >= c && q < c + kC && r > q) Mk[(long)r * np + q] = mk[h];
            }
            if (tid < kC) Mk[(long)(c + tid) * np + c + tid] = sdv[tid];
            __syncthreads();
        }
        if (failed) break;
        double* inv = A.dinv + (size_t)k * kTile * kTile;
        for (int q = tid; q < kTile * kTile; q += kSolveThreads) {
            const int r = q / kTile, c = q % kTile;
            inv[q] = c <= r ? Dinv[r][c] : 0.0;
        }
        // Forward substitution folded into the factorization: b_k has taken
        // every earlier tile's -L_kj y_j, so y_k = Dinv_k b_k now; the rows
        // below take -L_ik y_k during the trailing update.
        double yk = 0.0;
        if (tid < kTile) {
            for (int t = 0; t <= tid; ++t) yk += Dinv[tid][t] * x[k * kTile + t];
        }
        __syncthreads();
        if (tid < kTile) x[k * kTile + tid] = yk;
        // Panel: L_ik = A_ik Dinv^T, kStageRows rows at a time staged in LDS,
        // four elements per thread.  The raw rows of the next stage are read
        // into registers while the current one is computed (this stage writes
        // only its own rows).
        const bool in_lds = m <= kPanelRows;
        for (int r0 = 0; r0 < m; r0 += kStageRows) {
#pragma unroll
            for (int j = 0; j < kL; ++j) {
                const int q = tid + j * kSolveThreads;
                stage[(q / kTile) * kPanelStride + q % kTile] = raw[j];
            }
            __syncthreads();
            if (r0 + kStageRows < m) read_stage(r0 + kStageRows);
            // Column c of four rows per thread: each Dinv[c][t] is read once for
            // the four rows (same products and order per entry as a row-wise dot).
            const int c = tid % kTile;
            constexpr int kU = kStageRows * kTile / kSolveThreads;
            double acc[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) acc[u] = 0.0;
            for (int t = 0; t <= c; ++t) {
                const double dv = Dinv[c][t];
#pragma unroll
                for (int u = 0; u < kU; ++u) acc[u] += stage[(tid / kTile + u * (kSolveThreads / kTile)) * kPanelStride + t] * dv;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int rr = r0 + tid / kTile + u * (kSolveThreads / kTile);
                if (rr < m) {
                    A.M[(long)(R0 + rr) * np + k * kTile + c] = acc[u];
                    if (in_lds) panel[rr * kPanelStride + c] = acc[u];
                }
            }
            __syncthreads();
        }
        // Trailing update of the lower triangle, M[R][C] -= L[R] . L[C] for
        // R >= C >= R0: one wave per 32 x 32 tile.
        {
            const int tt = m / kTile;
            const int ntiles = tt * (tt + 1) / 2;
            const int wave = tid >> 6, lane = tid & 63;
            for (int tix = wave; tix < ntiles; tix += kSolveThreads / 64) {
                int ti = 0;
                while ((ti + 1) * (ti + 2) / 2 <= tix) ++ti;
                const int tj = tix - ti * (ti + 1) / 2;
                if (in_lds)
                    trailing_tile(A, (const double*)panel, kPanelStride, R0, ti, tj, lane, &D[0][0]);
                else
                    trailing_tile(A, (const double*)(A.M + (long)R0 * np + k * kTile), np, R0, ti, tj, lane, &D[0][0]);
            }
            // b_i -= L_ik y_k, one thread per panel row.
            for (int rr = tid; rr < m; rr += kSolveThreads) {
                double sacc = 0.0;
                for (int t = 0; t < kTile; ++t)
                    sacc += (in_lds ? panel[rr * kPanelStride + t] : A.M[(long)(R0 + rr) * np + k * kTile + t]) *
                            x[k * kTile + t];
                x[R0 + rr] -= sacc;
            }
        }
        __syncthreads();
    }
    if (failed) {
        if (tid == 0) A.state[0] = 1;
        return;
    }

    // Backward substitution L^T tau = y, tile by tile from the last: tau_k =
    // Dinv_k^T y_k (y_k has taken every later tile's share), then every earlier
    // entry c takes -sum over the tile's rows r of L[r][c] tau_r: reads along
    // rows of L, contiguous across threads.
    // A tile's reads of Dinv and of the L entries of each thread's first
    // column are issued together, before either is needed.
    for (int k = nt - 1; k >= 0; --k) {
        const double* inv = A.dinv + (size_t)k * kTile * kTile;
        constexpr int kI = kTile * kTile / kSolveThreads;
        double dv[kI];
#pragma unroll
        for (int j = 0; j < kI; ++j) dv[j] = inv[tid + j * kSolveThreads];
        const bool first = tid < k * kTile;
        double lr[kTile];
        if (first) {
#pragma unroll
            for (int r = 0; r < kTile; ++r) lr[r] = A.M[(long)(k * kTile + r) * np + tid];
        }
#pragma unroll
        for (int j = 0; j < kI; ++j) {
            const int q = tid + j * kSolveThreads;
            Dinv[q / kTile][q % kTile] = dv[j];
        }
        __syncthreads();
        double y = 0.0;
        if (tid < kTile) {
            for (int t = tid; t < kTile; ++t) y += Dinv[t][tid] * x[k * kTile + t];
        }
        __syncthreads();
        if (tid < kTile) x[k * kTile + tid] = y;
        __syncthreads();
        if (first) {
            double sacc = 0.0;
#pragma unroll
            for (int r = 0; r < kTile; ++r) sacc += lr[r] * x[k * kTile + r];
            x[tid] -= sacc;
        }
        for (int c = tid + kSolveThreads; c < k * kTile; c += kSolveThreads) {
            double sacc = 0.0;
#pragma unroll 8
            for (int r = 0; r < kTile; ++r) sacc += A.M[(long)(k * kTile + r) * np + c] * x[k * kTile + r];
            x[c] -= sacc;
        }
        __syncthreads();
    }

    apply_step<kSolveThreads>(A, x, red);
}

// ---------------------------------------------------------------- block-sparse solve
//
// The reduced system has one 7 x 7 block row per keyframe 1..N-1, and block
// (i, j) is non-zero only where an edge joins keyframes i and j.  In the
// natural (keyframe) order, Cholesky fills exactly the pairs of later
// neighbours of every eliminated block (a chain with a few loop closures fills
// little: the 32-keyframe benchmark graph's factor has 115 blocks of the 496
// in a dense lower triangle).  backend_pattern_kernel finds that pattern once
// per call; backend_sparse_solve_kernel factors only those blocks, in LDS,
// every iteration.  A pattern with more than kSpBlocks blocks takes the dense
// blocked solve instead (state[2]).

constexpr int kSpThreads = 256;
constexpr int kSpBlocks = 320;   // blocks of L in LDS: 320 x 392 B = 122.5 KB

// Bits j of word w (of a row's kPatWords words) with lo < j < hi.
__device__ __forceinline__ uint32_t bits_between(int w, int lo, int hi) {
    const long b0 = 32L * w;
    const uint64_t below_hi = hi <= b0 ? 0ull : (hi >= b0 + 32 ? 0xffffffffull : ((1ull << (hi - b0)) - 1ull));
    const uint64_t above_lo = lo < b0 ? 0xffffffffull : (lo >= b0 + 31 ? 0ull : (0xffffffffull << (lo - b0 + 1)));
    return (uint32_t)(below_hi & above_lo & 0xffffffffull);
}

// One workgroup, once per call: the lower block pattern of L after symbolic
// elimination in keyframe order (diagonal, every in-range edge between
// keyframes 1..N-1, then for each block column k every pair of its later
// non-zero rows), the slot of each block row's first block, and whether the
// factor fits the sparse solve.
__global__ void __launch_bounds__(kSpThreads) backend_pattern_kernel(BackendArgs A) {
    __shared__ uint32_t rows[M3S_MAX_KEYFRAMES * kPatWords];
    __shared__ uint32_t colm[kPatWords];
    __shared__ int32_t cnt[M3S_MAX_KEYFRAMES];
    const int nb = A.N - 1, tid = threadIdx.x;
    for (int i = tid; i < nb * kPatWords; i += kSpThreads) rows[i] = 0u;
    __syncthreads();
    for (int i = tid; i < nb; i += kSpThreads) atomicOr(&rows[i * kPatWords + (i >> 5)], 1u << (i & 31));
    for (int e = tid; e < A.E; e += kSpThreads) {
        const int ei = A.edges[2 * e], ej = A.edges[2 * e + 1];
        if (!edge_in_range(ei, ej, A.N) || ei == ej || ei == 0 || ej == 0) continue;
        const int a = max(ei, ej) - 1, b = min(ei, ej) - 1;
        atomicOr(&rows[a * kPatWords + (b >> 5)], 1u << (b & 31));
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (tid < kPatWords) colm[tid] = 0u;
        __syncthreads();
        for (int i = k + 1 + tid; i < nb; i += kSpThreads)
            if ((rows[i * kPatWords + (k >> 5)] >> (k & 31)) & 1u) atomicOr(&colm[i >> 5], 1u << (i & 31));
        __syncthreads();
        // Row x of the column takes every other row z of the column, k < z < x
        // (one writer per row).
        for (int x = k + 1 + tid; x < nb; x += kSpThreads) {
            if (!((colm[x >> 5] >> (x & 31)) & 1u)) continue;
            for (int w = 0; w < kPatWords; ++w) rows[x * kPatWords + w] |= colm[w] & bits_between(w, k, x);
        }
        __syncthreads();
    }
    for (int i = tid; i < nb; i += kSpThreads) {
        int c = 0;
        for (int w = 0; w < kPatWords; ++w) {
            A.pat[i * kPatWords + w] = rows[i * kPatWords + w];
            c += __popc(rows[i * kPatWords + w]);
        }
        cnt[i] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int i = 0; i < nb; ++i) {
            A.row_start[i] = t;
            t += cnt[i];
        }
        A.row_start[nb] = t;
        A.state[2] = t > kSpBlocks ? 1 : 0;
    }
}

// One workgroup per iteration: the block-sparse Cholesky of the assembled
// system over the pattern, the forward substitution folded in, the backward
// substitution, and the pose updates.  Per block column k, three barriers:
//   1. every lane factors L_kk = chol(A_kk) and forms L_kk^-1 in registers
//      (the same operations in every lane, so a block that is not positive
//      definite stops every lane alike), and y_k <- L_kk^-1 y_k; the later
//      rows of the column are listed in ascending order;
//   2. one lane per row a of each listed block: L_xk[a] <- A_xk[a] L_kk^-T,
//      then y_x[a] -= L_xk[a] . y_k;
//   3. one lane per entry of each listed pair x >= z: L_xz -= L_xk L_zk^T.
// L_kk^-1 replaces L_kk for the backward substitution L^T x = y, which one
// wave runs from the last block row up (x_k = L_kk^-T (y_k - sum_i L_ik^T x_i)).
__global__ void __launch_bounds__(kSpThreads) backend_sparse_solve_kernel(BackendArgs A) {
    __shared__ double Lb[kSpBlocks * 49];
    __shared__ double xs[kMaxDim];
    __shared__ uint32_t rows[M3S_MAX_KEYFRAMES * kPatWords];
    __shared__ int32_t rstart[M3S_MAX_KEYFRAMES];
    __shared__ uint8_t si[kSpBlocks], sj[kSpBlocks];
    __shared__ int32_t col[M3S_MAX_KEYFRAMES];
    __shared__ int32_t cslot[M3S_MAX_KEYFRAMES];  // slot of block (col[p], k)
    __shared__ uint64_t wb[kSpThreads / 64];
    __shared__ double red[kSpThreads / 64];
    if (A.state[0] || A.state[2]) return;
    const int nb = A.N - 1, np = A.np, tid = threadIdx.x;
    for (int i = tid; i < nb * kPatWords; i += kSpThreads) rows[i] = A.pat[i];
    for (int i = tid; i <= nb; i += kSpThreads) rstart[i] = A.row_start[i];
    for (int i = tid; i < A.n; i += kSpThreads) xs[i] = A.rhs[i];
    __syncthreads();
    const int nblk = rstart[nb];
    // Block (si[s], sj[s]) of every slot s, row-major.
    for (int i = tid; i < nb; i += kSpThreads) {
        int sl = rstart[i];
        for (int w = 0; w < kPatWords; ++w) {
            uint32_t m = rows[i * kPatWords + w];
            while (m) {
                const int j = 32 * w + __builtin_ctz(m);
                m &= m - 1u;
                si[sl] = (uint8_t)i;
                sj[sl] = (uint8_t)j;
                ++sl;
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < nblk * 49; q += kSpThreads) {
        const int sl = q / 49, e = q - 49 * (q / 49), a = e / 7, b = e - 7 * (e / 7);
        Lb[q] = A.M[(long)(7 * si[sl] + a) * np + 7 * sj[sl] + b];
    }
    __syncthreads();
    // Slot of block (i, j), j <= i, present in the pattern.
    auto slot = [&](int i, int j) -> int {
        int sl = rstart[i];
        for (int w = 0; w < (j >> 5); ++w) sl += __popc(rows[i * kPatWords + w]);
        return sl + __popc(rows[i * kPatWords + (j >> 5)] & ((1u << (j & 31)) - 1u));
    };
    const int wave = tid >> 6, lane = tid & 63;
    bool failed = false;
    for (int k = 0; k < nb; ++k) {
        // 1. L_kk and its inverse in registers (lower triangles), y_k.
        const double* Dk = Lb + 49 * (rstart[k + 1] - 1);  // the diagonal is row k's last block
        double L[7][7], Li[7][7], yk[7], isd[7];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            double d = Dk[7 * j + j];
#pragma unroll
            for (int m = 0; m < j; ++m) d -= L[j][m] * L[j][m];
            bad = bad || !(d > 0.0) || !isfinite(d);
            // 1/sqrt(d): hardware estimate and two Newton steps (no fp64
            // division or square root in the chain).
            double is = __builtin_amdgcn_rsq(d);
            is = is * fma(-0.5 * d * is, is, 1.5);
            is = is * fma(-0.5 * d * is, is, 1.5);
            L[j][j] = d * is;
            isd[j] = is;
#pragma unroll
            for (int i = j + 1; i < 7; ++i) {
                double v = Dk[7 * i + j];
#pragma unroll
                for (int m = 0; m < j; ++m) v -= L[i][m] * L[j][m];
                L[i][j] = v * is;
            }
        }
        if (bad) {
            failed = true;
            break;
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            Li[i][i] = isd[i];
#pragma unroll
            for (int j = 0; j < i; ++j) {
                double v = 0.0;
#pragma unroll
                for (int m = j; m < i; ++m) v += L[i][m] * Li[m][j];
                Li[i][j] = -v * Li[i][i];
            }
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m <= i; ++m) v += Li[i][m] * xs[7 * k + m];
            yk[i] = v;
        }
        // Later rows x of column k, ascending: one ballot per wave.
        const int xr = tid;
        const bool in_col = xr > k && xr < nb && ((rows[xr * kPatWords + (k >> 5)] >> (k & 31)) & 1u);
        const uint64_t bal = __ballot(in_col);
        if (lane == 0) wb[wave] = bal;
        __syncthreads();
        int ncol = 0, before = 0;
#pragma unroll
        for (int w = 0; w < kSpThreads / 64; ++w) {
            const int c = __popcll(wb[w]);
            if (w < wave) before += c;
            ncol += c;
        }
        if (in_col) {
            const int pos = before + __popcll(bal & ((1ull << lane) - 1ull));
            col[pos] = xr;
            cslot[pos] = slot(xr, k);
        }
        // The diagonal slot keeps L_kk^-1 (its lower triangle, the only part
        // the backward substitution reads) and y_k is final: one lane writes
        // both from registers with fixed offsets.
        if (tid == 0) {
            double* dk = Lb + 49 * (rstart[k + 1] - 1);
#pragma unroll
            for (int i = 0; i < 7; ++i) {
#pragma unroll
                for (int j = 0; j <= i; ++j) dk[7 * i + j] = Li[i][j];
                xs[7 * k + i] = yk[i];
            }
        }
        __syncthreads();
        // 2. Panel rows and the forward substitution.
        for (int q = tid; q < 7 * ncol; q += kSpThreads) {
            const int x = col[q / 7], a = q - 7 * (q / 7);
            double* row = Lb + 49 * cslot[q / 7] + 7 * a;
            double r[7], out[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) r[c] = row[c];
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < 7; ++b) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c <= b; ++c) v += r[c] * Li[b][c];
                out[b] = v;
                acc += v * yk[b];
            }
#pragma unroll
            for (int b = 0; b < 7; ++b) row[b] = out[b];
            xs[7 * x + a] -= acc;
        }
        __syncthreads();
        // 3. Trailing update of every listed pair x >= z.
        const int npair = ncol * (ncol + 1) / 2;
        for (int q = tid; q < 49 * npair; q += kSpThreads) {
            const int p = q / 49, e = q - 49 * (q / 49), a = e / 7, b = e - 7 * (e / 7);
            int xi = 0;
            while ((xi + 1) * (xi + 2) / 2 <= p) ++xi;
            const int zi = p - xi * (xi + 1) / 2;
            const int x = col[xi], z = col[zi];
            const double* lx = Lb + 49 * cslot[xi] + 7 * a;
            const double* lz = Lb + 49 * cslot[zi] + 7 * b;
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 7; ++c) v += lx[c] * lz[c];
            Lb[49 * slot(x, z) + e] -= v;
        }
        __syncthreads();
    }
    if (failed) {
        if (tid == 0) A.state[0] = 1;
        return;
    }
    // Backward substitution in wave 0, from the last block row up: every lane
    // forms x_k = L_kk^-T y_k (y_k has taken every later row's share), then
    // one lane per off-diagonal block (k, j) of row k (its slots are
    // consecutive) takes y_j -= L_kj^T x_k.  Row k is the only writer of those
    // y_j in its step, and the wave's LDS accesses complete in order.
    if (wave == 0) {
        for (int k = nb - 1; k >= 0; --k) {
            const int s0 = rstart[k], sd = rstart[k + 1] - 1;  // first and diagonal slot of row k
            const double* inv = Lb + 49 * sd;
            double yv[7], xk[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) yv[c] = xs[7 * k + c];
#pragma unroll
            for (int b = 0; b < 7; ++b) {
                double v = 0.0;
#pragma unroll
                for (int c = b; c < 7; ++c) v += inv[7 * c + b] * yv[c];
                xk[b] = v;
            }
            if (lane < 7) {
                double v = 0.0;
#pragma unroll
                for (int b = 0; b < 7; ++b) if (b == lane) v = xk[b];
                xs[7 * k + lane] = v;
            }
            for (int sl = s0 + lane; sl < sd; sl += 64) {
                const int j = sj[sl];
                const double* blk = Lb + 49 * sl;
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    double v = 0.0;
#pragma unroll
                    for (int a = 0; a < 7; ++a) v += blk[7 * a + c] * xk[a];
                    xs[7 * j + c] -= v;
                }
            }
        }
    }
    __syncthreads();
    apply_step<kSpThreads>(A, xs, red);
}

__global__ void __launch_bounds__(256) backend_finish_kernel(BackendArgs A) {
    const int t = threadIdx.x + blockIdx.x * blockDim.x;
    if (t < 12 * A.N) A.T_out[t] = (float)A.T64[t];
    if (t == 0 && A.info) {
        double cost = 0.0, count = 0.0;
        for (int e = 0; e < A.E; ++e) {
            if (!edge_in_range(A.edges[2 * e], A.edges[2 * e + 1], A.N)) continue;
            cost += A.edge_sys[(size_t)e * kStride + 35];
            count += A.edge_sys[(size_t)e * kStride + 36];
        }
        A.info[0] = (float)cost;
        A.info[1] = (float)count;
        A.info[2] = (float)A.state[1];
        A.info[3] = (float)A.stat[0];
    }
}

// Workspace layout.
struct BackendLayout {
    size_t T64, Trel, edge_sys, edge_blk, partials, state, stat, M, rhs, dinv, pat, row_start, total;
};

int padded_dim(int N) { return (7 * (N - 1) + kTile - 1) / kTile * kTile; }

BackendLayout backend_layout(int N, int HW, int E) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int bpe = backend_blocks_per_edge(HW);
    const size_t np = padded_dim(N);
    BackendLayout L;
    size_t o = 0;
    L.T64 = o;      o = al(o + sizeof(double) * 12 * N);
    L.Trel = o;     o = al(o + sizeof(float) * 12 * E);
    L.edge_sys = o; o = al(o + sizeof(double) * kStride * E);
    L.edge_blk = o; o = al(o + sizeof(double) * kBlk * E);
    L.partials = o; o = al(o + sizeof(float) * kStride * (size_t)bpe * E);
    L.state = o;    o = al(o + sizeof(int32_t) * 3);
    L.stat = o;     o = al(o + sizeof(double) * 2);
    L.M = o;        o = al(o + sizeof(double) * np * np);
    L.rhs = o;      o = al(o + sizeof(double) * np);
    L.dinv = o;     o = al(o + sizeof(double) * np * kTile);
    L.pat = o;      o = al(o + sizeof(uint32_t) * kPatWords * (size_t)N);
    L.row_start = o; o = al(o + sizeof(int32_t) * (size_t)N);
    L.total = o;
    return L;
}

}  // namespace

int backend_blocks_per_edge(int HW) {
    const int b = (HW + kThreads * kMatchesPerLane - 1) / (kThreads * kMatchesPerLane);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

size_t backend_workspace_bytes(int N, int HW, int E) { return backend_layout(N, HW, E).total; }

hipError_t launch_backend(int N, int HW, int E, const float* Xc, const float* Q, const int32_t* edges,
                          const int32_t* idx, const uint8_t* valid, float q_min, float sigma_ray, float sigma_dist,
                          float huber, int iters, double step_tol, float* T, float* info, void* ws, hipStream_t s) {
    const BackendLayout L = backend_layout(N, HW, E);
    char* w = reinterpret_cast<char*>(ws);
    BackendArgs A;
    A.N = N; A.HW = HW; A.E = E;
    A.blocks_per_edge = backend_blocks_per_edge(HW);
    A.n = 7 * (N - 1);
    A.np = padded_dim(N);
    A.Xc = Xc; A.Q = Q; A.edges = edges; A.idx = idx; A.valid = valid;
    A.q_min = (double)q_min;
    A.q_minf = q_min;
    A.rw = robust_weights(sigma_ray, sigma_dist, huber);
    A.step_tol = step_tol;
    A.T64 = reinterpret_cast<double*>(w + L.T64);
    A.Trel = reinterpret_cast<float*>(w + L.Trel);
    A.edge_sys = reinterpret_cast<double*>(w + L.edge_sys);
    A.edge_blk = reinterpret_cast<double*>(w + L.edge_blk);
    A.partials = reinterpret_cast<float*>(w + L.partials);
    A.state = reinterpret_cast<int32_t*>(w + L.state);
    A.stat = reinterpret_cast<double*>(w + L.stat);
    A.M = reinterpret_cast<double*>(w + L.M);
    A.rhs = reinterpret_cast<double*>(w + L.rhs);
    A.dinv = reinterpret_cast<double*>(w + L.dinv);
    A.pat = reinterpret_cast<uint32_t*>(w + L.pat);
    A.row_start = reinterpret_cast<int32_t*>(w + L.row_start);
    A.T_out = T;
    A.info = info;
    const dim3 grid(A.blocks_per_edge, E);
    backend_init_kernel<<<(12 * N + 255) / 256, 256, 0, s>>>(T, A.T64, N, A.state, A.stat);
    backend_relpose_kernel<<<(E + 255) / 256, 256, 0, s>>>(A);
    backend_pattern_kernel<<<1, kSpThreads, 0, s>>>(A);
    for (int it = 0; it <= iters; ++it) {
        const int final_pass = it == iters ? 1 : 0;
        timer_begin("backend_accum", s);
        backend_accum_kernel<<<grid, kThreads, 0, s>>>(A, final_pass);
        timer_end(s);
        timer_begin("backend_edge", s);
        backend_edge_kernel<<<E, kThreads, 0, s>>>(A, final_pass);
        timer_end(s);
        if (final_pass) break;
        timer_begin("backend_solve", s);
        backend_assemble_kernel<<<N, kAsmThreads, 0, s>>>(A);
        backend_sparse_solve_kernel<<<1, kSpThreads, 0, s>>>(A);
        backend_solve_kernel<<<1, kSolveThreads, 0, s>>>(A);
        timer_end(s);
    }
    backend_finish_kernel<<<(12 * N + 255) / 256, 256, 0, s>>>(A);
    return hipGetLastError();
}

}  // namespace m3s
