/*
 * m3s.h -- C ABI of the MI355X (gfx950) projective pointmap matcher.
 *
 * The library implements the pointmap matching of MASt3R-SLAM (Murai,
 * Dexheimer, Davison, CVPR 2025, arXiv 2412.12392), Sec. 3.2:
 *
 *   m_{i,j} = M(X^i_i, X^j_i, D^i_i, D^j_i)
 *
 * For every pixel n of the query pointmap X^j_i (both pointmaps are expressed
 * in camera i, Sec. 3.1), it finds the pixel p of frame i whose normalised ray
 * psi(X^i_i(p)) best aligns with psi(x_n) by minimising the ray error of Eq. 2,
 * |psi([X^i_i]_p) - psi(x_n)|^2, with Levenberg-Marquardt (Sec. 3.2), reports
 * the residual angle of Eq. 3, refines the integer match to the best
 * descriptor dot product in a small window (Sec. 3.2, feature refinement), and
 * gates it by residual angle, match confidence sqrt(Q^i_i[m] Q^j_i[n])
 * (Sec. 3.3) and 3D distance (Sec. 3.2, occlusion and outlier handling).
 * A backward pass gives the implicit adjoint of the converged match, a
 * batched entry point matches many edges of a keyframe graph in one launch,
 * the tracking entry point solves a frame's Sim(3) pose from its matches and
 * fuses its pointmap into the keyframe's (Sec. 3.3), and the backend entry
 * point solves the keyframe poses over the whole graph (Sec. 3.5).
 *
 * Conventions shared by every entry point:
 *   - All array arguments are caller-owned DEVICE memory (HBM of the current
 *     HIP device), fp32 unless stated, row-major, pixel m = y * W + x.
 *     Pointmaps are H*W*3 (x, y, z interleaved); descriptors H*W*D;
 *     confidences H*W; pixel positions H*W*2 as (x = column, y = row).
 *   - Pixel centres are at integer coordinates; the match domain is
 *     [0, W-1] x [0, H-1].  H and W must be at least 2.
 *   - The library never keeps, frees or reallocates caller memory.  The
 *     workspace is caller-provided device memory of the size the matching
 *     *_workspace_bytes function reports; its contents need not be preserved
 *     between calls (except as stated for m3s_match_batched).
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream).  Arguments are validated on the host first: on any error
 *     nothing is enqueued and a status code is returned; m3s_last_error()
 *     then describes the problem (per calling thread).  Faults inside kernels
 *     surface when the caller synchronises the stream.
 *   - The library never aborts, exits or prints.
 */
#ifndef M3S_H
#define M3S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define M3S_VERSION 2
#define M3S_MAX_RADIUS 8      /* largest refine radius r */
#define M3S_MAX_ITER 1000     /* largest LM iteration count K */
#define M3S_MAX_DESC 64       /* largest descriptor dimension D */
#define M3S_MAX_PIXELS (1 << 26)  /* largest H * W of one frame (67,108,864 pixels) */
#define M3S_MAX_LEVELS 4      /* largest number of coarse-to-fine refine levels */
#define M3S_MAX_KEYFRAMES 128 /* largest number of keyframes of one backend solve */
#define M3S_MAX_EDGES 65535   /* largest number of edges of one backend solve */

typedef enum {
    M3S_OK = 0,
    M3S_ERR_NULL = 1,         /* a required pointer is NULL */
    M3S_ERR_SHAPE = 2,        /* H, W < 2, H * W > M3S_MAX_PIXELS, D out of [1, M3S_MAX_DESC] */
    M3S_ERR_PARAM = 3,        /* a parameter out of its documented range */
    M3S_ERR_WORKSPACE = 4,    /* workspace NULL, misaligned (256 B) or too small */
    M3S_ERR_HIP = 5,          /* a HIP runtime call failed */
    M3S_ERR_UNSUPPORTED = 6,  /* device is not gfx950, or an unsupported flag */
    M3S_STATUS_RESERVED = 0x7fffffff  /* not returned; keeps any int32 a valid m3s_status value */
} m3s_status;

/*
 * Matching parameters (Sec. 3.2 and 3.3).  m3s_default_params fills the
 * values of the paper's setting: K = 10 iterations ("within 10 iterations"),
 * lambda 1e-8, refine radius 3 with one level, confidence gate 1.5,
 * residual-angle gate 1e-4 rad and no 3D-distance gate.
 */
typedef struct {
    int32_t max_iter;       /* K in [0, M3S_MAX_ITER]: LM iterations, run exactly (no early exit) */
    float   lambda_init;    /* initial Levenberg damping, finite and > 0 */
    int32_t refine_radius;  /* r in [0, M3S_MAX_RADIUS]: window (2r+1)^2; 0 = round(p*) */
    int32_t refine_levels;  /* L in [1, M3S_MAX_LEVELS]: coarse-to-fine levels of spacing 2^(L-1)..1 */
    float   conf_min;       /* q_min: valid needs sqrt(Qii[idx] * Qji[n]) >= conf_min (if Q given); finite */
    float   max_theta;      /* valid needs residual angle <= max_theta (rad); >= 0, may be +inf */
    float   max_dist;       /* valid needs |Xii[idx] - Xji[n]| <= max_dist; > 0, +inf disables the gate */
} m3s_params;

/* One matching problem: reference frame i and query pointmap X^j_i, same H x W. */
typedef struct {
    int32_t H, W, D;
    const float *Xii;       /* [H*W*3] reference pointmap X^i_i (required) */
    const float *Xji;       /* [H*W*3] query pointmap X^j_i in camera i (required) */
    const float *Dii;       /* [H*W*D] reference descriptors D^i_i (required) */
    const float *Dji;       /* [H*W*D] query descriptors D^j_i (required) */
    const float *Qii;       /* [H*W] descriptor confidence Q^i_i, or NULL */
    const float *Qji;       /* [H*W] descriptor confidence Q^j_i, or NULL (both or neither) */
    const float *p_init;    /* [H*W*2] initial pixel per query, or NULL for the identity mapping */
} m3s_pair;

/*
 * Per-query outputs.  p, idx and valid are required; theta and xhat may be
 * NULL.  A query with a non-finite or zero point, or a non-finite initial
 * pixel, gets idx = -1, valid = 0, theta = +inf and p = its clamped initial
 * pixel (0 if that is non-finite).
 */
typedef struct {
    float   *p;             /* [H*W*2] continuous match p* before refinement, (x, y) */
    int32_t *idx;           /* [H*W]   refined match, linear pixel index in frame i, or -1 */
    uint8_t *valid;         /* [H*W]   1 if the match passes every gate, else 0 */
    float   *theta;         /* [H*W]   residual angle at p* in radians (Eq. 3), or NULL */
    float   *xhat;          /* [H*W*3] X^i_i sampled bilinearly at p*, or NULL */
} m3s_outputs;

/* One edge of a batch: its pair, its outputs, and optional per-edge K and r (< 0: use the common ones);
   the refine levels are the common ones. */
typedef struct {
    m3s_pair    in;
    m3s_outputs out;
    int32_t     max_iter;
    int32_t     refine_radius;
} m3s_edge;

/* Fills *params with the defaults listed above.  NULL is ignored. */
void m3s_default_params(m3s_params *params);

/*
 * Workspace bytes m3s_match_fwd needs for this pair (0 on invalid shapes).
 * The workspace holds the ray image of X^i_i and its gradient images.
 */
size_t m3s_workspace_bytes(const m3s_pair *pair, const m3s_params *params);

/*
 * m3s_match_fwd -- match every pixel of pair->Xji (Sec. 3.2, Eq. 2 and 3;
 * gates of Sec. 3.2 and 3.3).  Steps, all on the GPU:
 *   ray image R = X^i_i / |X^i_i| and its central-difference gradient images;
 *   per query: target ray t = x / |x|, start at p_init or the query's own
 *   pixel, K Levenberg-Marquardt iterations on |psi_hat(p) - t|^2 with the
 *   bilinearly sampled, renormalised ray psi_hat, damping lambda I (x10 on a
 *   rejected step, /10 on an accepted one), every iterate clamped to the
 *   image (a coordinate on its bound whose step points outward is held);
 *   residual angle 2 asin(|e| / 2); refine to the first maximum of the raw
 *   descriptor dot product over the (2r+1)^2 window around round(p*), or
 *   coarse to fine over L levels of spacing 2^(L-1), ..., 1, each around the
 *   previous level's best (Sec. 3.2, feature refinement); gates.
 * ws must be 256-byte aligned device memory of >= m3s_workspace_bytes().
 */
m3s_status m3s_match_fwd(const m3s_pair *pair, const m3s_params *params, const m3s_outputs *out,
                         void *ws, size_t ws_bytes, void *stream);

/*
 * m3s_match_fwd_noalloc -- m3s_match_fwd with no workspace argument, for
 * callers that cannot allocate device memory (code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The ray
 * records live in a static device array of the library, one copy per GPU,
 * sized for M3S_NOALLOC_MAX_PIXELS pixels (36 B each: 9 MiB) and held until
 * the process ends; the call itself allocates nothing (no hipMalloc, no
 * hipFree, no events even with timing enabled).  H * W above the limit
 * returns M3S_ERR_SHAPE.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (several streams or host threads at once) race and
 * must be serialised by the caller.  The caller still provides the inputs
 * and outputs.  Results equal m3s_match_fwd's bit for bit.
 */
#define M3S_NOALLOC_MAX_PIXELS (1 << 18)
m3s_status m3s_match_fwd_noalloc(const m3s_pair *pair, const m3s_params *params, const m3s_outputs *out,
                                 void *stream);

/*
 * m3s_match_bwd -- implicit adjoint of the converged match (no counterpart in
 * the paper).  Given the forward's p and valid, and upstream gradients
 * grad_p [H*W*2] (required) and grad_xhat [H*W*3] (or NULL), writes
 * grad_Xii and grad_Xji [H*W*3] each (overwritten) for the dependence of p*
 * and xhat on the two pointmaps.  At p* the ray residual vanishes, so with
 * Je = d psi_hat / d p (exact derivative of the bilinear ray sample) the
 * adjoint solves (Je^T Je) mu = g, v = Je mu, and scatters
 * grad_Xji[n] = N(x_n) v and grad_Xii[c] -= w_c N(X^i_i[c]) v / |r|, with
 * N(X) = (I - X X^T/|X|^2)/|X| (Supp. A, Eq. norm_jac), plus the bilinear
 * weights of grad_xhat into the four corners of p*.  Invalid queries
 * contribute nothing.  grad_Xii sums the terms of each 16 x 16 query tile in
 * 64-bit fixed point (exact, independent of their order) and adds the tiles'
 * sums with fp32 atomics, so its rounding may differ between runs.  No
 * workspace is needed.
 */
m3s_status m3s_match_bwd(const m3s_pair *pair, const m3s_outputs *fwd,
                         const float *grad_p, const float *grad_xhat,
                         float *grad_Xii, float *grad_Xji, void *stream);

/*
 * m3s_match_bwd_batched -- m3s_match_bwd over n_edges edges (for example the
 * edges just matched by m3s_match_batched) in two launches: one zeroes every
 * grad_Xii, then one persistent launch works through the 16 x 16 query tiles
 * of all edges.  With M3S_BWD_ACCUMULATE in flags there is no zeroing launch:
 * the gradients are added to grad_Xii's contents (gradient accumulation, for
 * example several edges of one keyframe into one buffer, or a buffer the
 * caller cleared on another stream while the forward ran); grad_Xji is still
 * overwritten.  `edges` is a HOST array, copied into the workspace on
 * `stream` before the launches (the caller may reuse it when the call
 * returns).  grad_Xji equals m3s_match_bwd's bit for bit; grad_Xii equals it
 * up to the order of the fp32 atomic additions.  With M3S_BATCH_GRAPH the two
 * launches are captured into a hipGraph keyed by (device, workspace address,
 * edge shapes) and replayed.  The call cannot itself be captured into a
 * caller's graph (it returns M3S_ERR_UNSUPPORTED on a capturing stream).
 * Calls that share a workspace must not overlap.
 */
typedef struct {
    int32_t H, W;
    const float   *Xii, *Xji;      /* [H*W*3] the edge's pointmaps */
    const float   *p;              /* [H*W*2] the forward's p */
    const uint8_t *valid;          /* [H*W]   the forward's valid */
    const float   *grad_p;         /* [H*W*2] required */
    const float   *grad_xhat;      /* [H*W*3] or NULL */
    float         *grad_Xii;       /* [H*W*3] overwritten (added to with M3S_BWD_ACCUMULATE) */
    float         *grad_Xji;       /* [H*W*3] overwritten */
} m3s_bwd_edge;
size_t m3s_bwd_batched_workspace_bytes(int32_t n_edges);
m3s_status m3s_match_bwd_batched(const m3s_bwd_edge *edges, int32_t n_edges, uint32_t flags, void *ws,
                                 size_t ws_bytes, void *stream);

/*
 * Keyframe statistics of one match set (Sec. 3.4: tracking adds a keyframe
 * when the number of valid matches or of distinct matched keyframe pixels
 * falls below a fraction of the pixels).  From the forward's idx and valid
 * (H*W queries matched into an H x W reference frame), writes the DEVICE
 * array counts[2] = {number of valid queries, number of distinct idx among
 * them} (overwritten).  ws: 256-byte aligned device memory of at least
 * m3s_stats_workspace_bytes(H, W) (a bitmap of the reference pixels).
 */
size_t m3s_stats_workspace_bytes(int32_t H, int32_t W);
m3s_status m3s_match_stats(const m3s_outputs *fwd, int32_t H, int32_t W, int32_t *counts,
                           void *ws, size_t ws_bytes, void *stream);

/*
 * Tracking pose solve (Sec. 3.3).  The current frame f is matched to the last
 * keyframe k with the keyframe's pixels as queries (m3s_match_fwd with
 * Xii = X^f_f and Xji = X^k_f), so idx[n] is the frame pixel m of keyframe
 * pixel n.  The pose T_kf = [sR | t] (Sim(3), maps frame points into the
 * keyframe) is refined by Gauss-Newton with robust weights recomputed at
 * every iteration (Eq. gauss_newton) over every valid match with
 * q = sqrt(Qf[m] Qk[n]) > q_min:
 *   ray residual      psi(T Xf[m]) - psi(Xk[n])    weight q / sigma_ray^2
 *   distance residual |T Xf[m]| - |Xk[n]|           weight q / sigma_dist^2
 * each weight times the Huber weight of the block's whitened norm
 * |r| sqrt(q) / sigma (width `huber`); Jacobians w.r.t. a left perturbation
 * tau = (v, omega, sigma) (Supp. A); the 7x7 normal equations are summed,
 * solved by Cholesky in fp64 (a step whose system is not positive definite
 * is skipped) and applied as T <- Exp(tau) o T (Eq. 1).  Residuals and
 * Jacobians are evaluated in fp32, the normal equations summed in fp32 per
 * workgroup and in fp64 across workgroups; the confidence gate is decided in
 * fp64.
 */
typedef struct {
    int32_t iters;          /* Gauss-Newton iterations, run exactly, in [0, M3S_MAX_ITER] */
    float   q_min;          /* confidence gate: a match needs q > q_min; finite */
    float   sigma_ray;      /* ray residual sigma, > 0; +inf drops the ray residual */
    float   sigma_dist;     /* distance residual sigma, > 0; +inf drops the distance residual */
    float   huber;          /* Huber width on the whitened norm, > 0; +inf = plain least squares */
} m3s_track_params;

/* One tracking problem: keyframe k and current frame f, same H x W. */
typedef struct {
    int32_t H, W;
    const float   *Xk;      /* [H*W*3] keyframe points X~^k_k (the measurements, required) */
    const float   *Xf;      /* [H*W*3] frame points X^f_f (required) */
    const int32_t *idx;     /* [H*W]   match of keyframe pixel n: frame pixel in [0, H*W), or < 0 (required) */
    const uint8_t *valid;   /* [H*W]   match flags (required) */
    const float   *Qf;      /* [H*W]   frame confidence Q^f_f (required) */
    const float   *Qk;      /* [H*W]   keyframe confidence Q^k_k (required) */
} m3s_track_problem;

/* Fills *params with q_min 1.5, sigma_ray 0.003, sigma_dist 0.1, Huber 1.345, 10 iterations.  NULL is ignored. */
void m3s_default_track_params(m3s_track_params *params);

/* Workspace bytes m3s_track_pose needs for an H x W keyframe (0 on invalid shapes). */
size_t m3s_track_workspace_bytes(int32_t H, int32_t W);

/*
 * m3s_track_pose -- `iters` Gauss-Newton iterations from the pose in T.
 *   T     DEVICE float[12], row-major 3x4 [sR | t]: the initial pose on entry,
 *         the refined pose when the stream reaches the end of the call.
 *   info  DEVICE float[4] or NULL: {robust cost at the final pose, number of
 *         matches used there, number of iterations whose system was solved,
 *         norm of the last applied step}.
 *   ws    256-byte aligned DEVICE memory of >= m3s_track_workspace_bytes();
 *         calls that share a workspace must not overlap.
 * Matches with idx outside [0, H*W), non-finite or zero points are skipped.
 * Two launches per iteration plus three, no host synchronisation: the call can
 * be captured into a hipGraph.
 */
m3s_status m3s_track_pose(const m3s_track_problem *prob, const m3s_track_params *params, float *T, float *info,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * Canonical pointmap fusion (Sec. 3.3, Eq. 8): after the pose solve, every
 * keyframe pixel n takes the running confidence-weighted average
 *   Xc[n] <- (Cc[n] Xc[n] + C[n] (T X[n])) / (Cc[n] + C[n]),   Cc[n] <- Cc[n] + C[n]
 * of its canonical point and the frame's prediction of it moved into the
 * keyframe by T = T_kf.  A pixel whose summed confidence is not positive
 * keeps its point.  fp32; Cc is the fp32 sum exactly rounded.
 */
typedef struct {
    int32_t H, W;
    float       *Xc;        /* [H*W*3] canonical pointmap X~^k_k, updated in place (required) */
    float       *Cc;        /* [H*W]   its summed confidence C~^k_k, updated in place (required) */
    const float *X;         /* [H*W*3] the frame's prediction X^k_f of the keyframe's points (required) */
    const float *C;         /* [H*W]   its confidence C^k_f (required) */
} m3s_fuse_problem;

/*
 * m3s_fuse_pointmap -- Eq. 8 over every pixel.  T is a DEVICE float[12]
 * (row-major 3x4 [sR | t]), read when the stream reaches the call, so it may
 * be the T that m3s_track_pose just wrote on the same stream.  Arrays must be
 * 4-byte aligned; 16-byte aligned arrays take the vectorised path.  No
 * workspace.
 */
m3s_status m3s_fuse_pointmap(const m3s_fuse_problem *prob, const float *T, void *stream);

/*
 * Backend optimisation (Sec. 3.5).  N keyframes of one H x W resolution with
 * world poses T_WC[k] (Sim(3), 3x4 [sR | t]) and canonical pointmaps; E edges
 * (i, j), each with the matches of keyframe j's pixels into keyframe i
 * (m3s_match_fwd with Xii = X~^i_i and Xji = T_ij X~^j_j, so idx[n] is a pixel
 * of i).  Gauss-Newton on the global ray objective (Eq. backend_ray) plus the
 * small-weight distance term, over every valid match with
 * q = sqrt(Q[i][m] Q[j][n]) > q_min:
 *   ray residual      psi(T_ij Xc[j][n]) - psi(Xc[i][m])   weight q / sigma_ray^2
 *   distance residual |T_ij Xc[j][n]| - |Xc[i][m]|         weight q / sigma_dist^2
 * with T_ij = T_WC[i]^-1 T_WC[j], Huber weights as in m3s_track_pose, and the
 * world-pose Jacobians -J Ad(T_WC[i]^-1), J Ad(T_WC[i]^-1) (Supp. A).  Keyframe 0
 * holds the gauge.  The reduced 7(N-1) system is solved by a block-sparse
 * Cholesky factorisation in fp64 over 7 x 7 blocks in keyframe order (a dense
 * one when the factor's fill exceeds 320 blocks; the same solution either way)
 * and every other pose takes T_WC[k] <- Exp(tau_k) o T_WC[k] (Eq. 1).  The loop ends after
 * `iters` steps, once a step norm |tau| falls below step_tol (that step is
 * applied), or when the system is not positive definite (no step applied).
 * Residuals are evaluated in fp32 and summed per workgroup in fp32, per edge
 * and across edges in fp64; the confidence gate is decided in fp64.
 */
typedef struct {
    int32_t iters;          /* at most this many Gauss-Newton steps, in [0, M3S_MAX_ITER] */
    float   q_min;          /* confidence gate, finite */
    float   sigma_ray;      /* > 0; +inf drops the ray residual */
    float   sigma_dist;     /* > 0; +inf drops the distance residual */
    float   huber;          /* Huber width on the whitened norm, > 0; +inf = plain least squares */
    double  step_tol;       /* >= 0: stop once |tau| < step_tol (0: run all iterations); steps do not
                               fall below about 1e-7 (1 + |t|), the fp32 rounding of the relative poses */
} m3s_backend_params;

typedef struct {
    int32_t N, H, W;        /* keyframes (2 .. M3S_MAX_KEYFRAMES) and their common resolution */
    int32_t E;              /* edges, 1 .. M3S_MAX_EDGES */
    const float   *Xc;      /* [N*H*W*3] canonical pointmaps, keyframe-major (required) */
    const float   *Q;       /* [N*H*W]   per-keyframe confidences (required) */
    const int32_t *edges;   /* [E*2]     DEVICE (i, j) per edge; edges outside [0, N) are skipped (required) */
    const int32_t *idx;     /* [E*H*W]   per edge, the pixel of i matched to pixel n of j, or < 0 (required) */
    const uint8_t *valid;   /* [E*H*W]   per edge, match flags (required) */
} m3s_backend_problem;

/* Fills *params with the tracking defaults, 10 iterations and step_tol 0.  NULL is ignored. */
void m3s_default_backend_params(m3s_backend_params *params);

/* Workspace bytes m3s_backend_gn needs (0 on invalid sizes). */
size_t m3s_backend_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t E);

/*
 * m3s_backend_gn -- the Gauss-Newton loop above.
 *   T_WC  DEVICE float[N*12], the initial world poses on entry and the solved
 *         ones when the stream reaches the end of the call (keyframe 0 is
 *         written back unchanged).
 *   info  DEVICE float[4] or NULL: {robust cost at the final poses, matches
 *         used there, steps applied, norm of the last applied step}.
 *   ws    256-byte aligned DEVICE memory of >= m3s_backend_workspace_bytes();
 *         calls that share a workspace must not overlap.
 * 6 + 5 * iters launches on `stream`, no host synchronisation (a graph can
 * capture the call); after the loop has ended, the remaining launches return
 * at once.  The solve runs in one workgroup: the block pattern of the factor
 * is found once per call, and each iteration factors the pattern's blocks in
 * LDS, or, when they do not fit, factors the dense reduced system blocked in
 * 32 x 32 tiles.
 */
m3s_status m3s_backend_gn(const m3s_backend_problem *prob, const m3s_backend_params *params, float *T_WC,
                          float *info, void *ws, size_t ws_bytes, void *stream);

/* Flags of m3s_match_batched. */
#define M3S_BATCH_GRAPH    0x1u  /* capture the launch sequence in a hipGraph and replay it */
#define M3S_BATCH_AUTOTUNE 0x2u  /* time candidate launch shapes once per shape signature */
#define M3S_BWD_ACCUMULATE 0x4u  /* m3s_match_bwd_batched: add to grad_Xii instead of overwriting it */

/*
 * Workspace bytes m3s_match_batched needs for these edges (0 on invalid input):
 * the ray images of every edge, a device copy of the edge table and the
 * work-queue counter.
 */
size_t m3s_batched_workspace_bytes(const m3s_edge *edges, int32_t n_edges, const m3s_params *common);

/*
 * m3s_match_batched -- m3s_match_fwd over n_edges edges (the edges of a
 * keyframe graph, Sec. 3.4; matching every new edge is the per-keyframe
 * cost of Sec. 3.2) in one persistent launch.  Edges may differ in H, W, K
 * and r (D may differ too).  `edges` is a HOST array; it is copied into the
 * workspace on `stream` before the launch, so the caller may reuse it as
 * soon as the call returns.  Results equal those of m3s_match_fwd on each
 * edge bit for bit.  With M3S_BATCH_GRAPH the launch sequence is captured
 * into a hipGraph keyed by (device, workspace address, edge shapes) and
 * replayed on later calls with the same key; the edge table lives in the
 * workspace, so new pointers need no re-capture.  With M3S_BATCH_AUTOTUNE
 * the first call for a shape signature times candidate launch shapes (see
 * m3s_set_tune_cache; this first call synchronises the stream) and caches the
 * fastest; later calls with that signature, in this process or, with a cache
 * file, in another, are asynchronous.  Calls that share a
 * workspace must not overlap.  The call cannot itself be captured into a
 * caller's hipGraph (it copies the edge table from host memory before each
 * launch): on a capturing stream it returns M3S_ERR_UNSUPPORTED.
 */
m3s_status m3s_match_batched(const m3s_edge *edges, int32_t n_edges, const m3s_params *common,
                             uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* Launch shape the batched path used for its last call on this thread: workgroups, tile id. */
void m3s_batched_last_config(int32_t *grid, int32_t *tile_config);

/*
 * Diagnostics: launch override and fallback-path counters (for tests and
 * benchmarks; a production caller needs neither).
 *
 * m3s_debug_set_launch fixes the launch shape of later m3s_match_fwd and
 * m3s_match_batched calls made by the CALLING THREAD (NULL restores the
 * library's choice; -1 or 0 in a field keeps the library's choice for it):
 *   tile_config  0: 32x8, 1: 16x16, 2: 64x4 query tiles refining from global
 *                memory; 3: 16x16, 4: 32x8 with the refine region staged in LDS
 *                (fp32); 5: 16x16 with an fp16 pre-filter (the default); 6: 8x8
 *                one-wave tiles with the fp16 pre-filter;
 *   grid         workgroups of the persistent batched launch (> 0);
 *   xcd_remap    0 turns off the tile-to-XCD band mapping of the single-pair launch;
 *   ray_margin   margin in pixels (1..3, default 2) of the LM ray window the
 *                batched fp16 configuration stages around its queries' cells;
 *   lm_unroll    unroll factor (1 or 2) of its LM iteration loop.
 * An override also disables M3S_BATCH_AUTOTUNE.  Every configuration gives
 * the same output bits.  m3s_batched_last_launch reads back the launch the
 * calling thread's last m3s_match_batched used (xcd_remap -1).
 */
typedef struct {
    int32_t tile_config;
    int32_t grid;
    int32_t xcd_remap;
    int32_t ray_margin;
    int32_t lm_unroll;
} m3s_launch_config;
void m3s_debug_set_launch(const m3s_launch_config *cfg);
void m3s_batched_last_launch(m3s_launch_config *cfg);

/*
 * Autotuning cache on disk.  M3S_BATCH_AUTOTUNE times, once per batch shape,
 * every tile configuration at 1, 2, 4 and 8 workgroups per CU and then, for
 * the fp16 configuration, every ray-window margin and LM unroll at its best
 * grid, and keeps the fastest launch keyed by (device architecture, CU count,
 * shape signature of the edges).  m3s_set_tune_cache(path) loads the entries
 * of a cache file written earlier (a missing file is fine; a file of another
 * format or version returns M3S_ERR_PARAM and changes nothing) and from then
 * on writes every new result back to it (a temporary file renamed over the
 * old one).  NULL stops writing; the results already loaded stay.
 */
m3s_status m3s_set_tune_cache(const char *path);

/*
 * Counters of the fallback paths taken on the current device since the last
 * reset, each a 64-bit count of tiles (of queries for M3S_PATH_REFINE_QUERY):
 *   M3S_PATH_LM_GLOBAL      LM iterations 2..K read the ray records from global
 *                           memory because the tile's window exceeded the LDS cap;
 *   M3S_PATH_REFINE_GLOBAL  the refine scanned global memory exactly because the
 *                           tile's region exceeded LDS, held a value outside the
 *                           fp16 range, r > 5 or L > 1 (LDS tile configurations);
 *   M3S_PATH_REFINE_QUERY   a query's own descriptor norm was outside the fp16
 *                           range (fp16 configuration): exact global scan;
 *   M3S_PATH_BWD_DIRECT     a backward tile's corner window exceeded LDS, so its
 *                           gradients went to dL/dX^i_i by direct global atomics;
 *   M3S_PATH_REFINE_BANDS   a coarse-to-fine level's region exceeded LDS and was
 *                           staged and pre-filtered in fp16 in up to six bands of
 *                           whole rows (not a fallback: counted so that tests can
 *                           show the banded path ran).
 * Writes counts[M3S_PATH_COUNTERS] and, if reset != 0, zeroes the counters.
 * Synchronises the device.
 */
#define M3S_PATH_LM_GLOBAL     0
#define M3S_PATH_REFINE_GLOBAL 1
#define M3S_PATH_REFINE_QUERY  2
#define M3S_PATH_BWD_DIRECT    3
#define M3S_PATH_REFINE_BANDS  4
#define M3S_PATH_COUNTERS      8
m3s_status m3s_path_counters(int64_t *counts, int32_t reset);

/*
 * Kernel timing (off by default).  When enabled, the library records a pair of
 * hipEvents around every kernel it launches eagerly (and around each hipGraph
 * launch, as "batched_graph").  m3s_timing_read synchronises on the recorded
 * events and returns, for the kernel `name` ("prep", "fwd", "fill", "bwd",
 * "batched_prep" (with the reset of the work-queue counter), "batched_fwd",
 * "batched_graph", "batched_bwd_zero", "batched_bwd", "batched_bwd_graph",
 * "track_step" (one Gauss-Newton iteration: the previous system's solve and
 * the accumulation), "track_final", "fuse" (the vectorised launch),
 * "backend_accum", "backend_edge", "backend_solve"), the
 * summed duration in milliseconds and the number of launches since the last
 * reset.  Meant for benchmarks: the events cost a little time per launch.
 */
void m3s_timing_enable(int32_t on);
m3s_status m3s_timing_read(const char *name, double *total_ms, int64_t *launches);
void m3s_timing_reset(void);

/* Drops every cached hipGraph and autotuning result. */
void m3s_clear_caches(void);

/* Static description of a status code. */
const char *m3s_status_string(m3s_status status);

/* Details of the last error on the calling thread ("" if none). */
const char *m3s_last_error(void);

/* M3S_VERSION of the library. */
int32_t m3s_version(void);

#ifdef __cplusplus
}
#endif

#endif /* M3S_H */
