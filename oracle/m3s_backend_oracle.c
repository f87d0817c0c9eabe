/*
 * FP64 CPU oracle for the backend optimisation of MASt3R-SLAM (Sec. 3.5).
 *
 * TEST INFRASTRUCTURE ONLY (see m3s_oracle.c): shares no code with the HIP
 * library and is never linked into it.
 *
 * N keyframes share one H x W resolution; keyframe k has its canonical
 * pointmap Xc[k] (H*W*3), a per-pixel confidence Q[k] (H*W) and its world
 * pose T_WC[k] (Sim(3), row-major 3x4 [sR | t]).  Edge e = (i, j) holds the
 * matches of frame j's pixels into frame i (idx[e][n] = pixel m of i, with a
 * valid flag), as the matcher produces them with X^i_i as reference.
 *
 * Global ray objective (Eq. backend_ray) plus the small-weight distance term,
 * for every valid match with q = sqrt(Q[i][m] Q[j][n]) > q_min:
 *   x = T_ij Xc[j][n],  T_ij = T_WC[i]^-1 T_WC[j]
 *   r_ray  = psi(x) - psi(Xc[i][m])      (Supp. A: the transformed point minus
 *   r_dist = |x| - |Xc[i][m]|             the measured one, as in tracking)
 *   D r / D T_ij = [N(x), -[x]_x / |x|, 0] and [x^T / |x|, 0, |x|] (Supp. A)
 *   D r / D T_WC[i] = -(D r / D T_ij) Ad(T_WC[i]^-1),
 *   D r / D T_WC[j] =  (D r / D T_ij) Ad(T_WC[i]^-1)   (Supp. A, relative to
 *                                                       global pose)
 *   weights q / sigma^2 times the Huber weight of the whitened block norm,
 *   exactly as in the tracking oracle.
 * The 7N x 7N normal equations are summed match by match; the gauge is fixed
 * by holding keyframe 0 (its rows and columns are dropped); the reduced
 * system is solved by Cholesky and every other pose takes
 * T_WC[k] <- Exp(tau_k) o T_WC[k] (Eq. 1).  At most `iters` iterations; the
 * loop ends early once the step norm |tau| falls below step_tol (after that
 * step is applied), or when the system is not positive definite.
 *
 * Readings where the paper is silent: the match confidence comes from
 * per-keyframe confidence images; the convergence test is on |tau|; the
 * paper's sparse Cholesky is replaced by a dense one (same solution up to
 * rounding).  Adjoint of a Sim(3) T = [sR | t] on (v, omega, sigma):
 *   Ad(T) = [[sR, [t]_x R, -t], [0, R, 0], [0, 0, 1]].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* From m3s_track_oracle.c (same library). */
void oracle_sim3_exp(const double tau[7], double T[12]);

static void bk_skew(const double x[3], double S[3][3])
{
    S[0][0] = 0; S[0][1] = -x[2]; S[0][2] = x[1];
    S[1][0] = x[2]; S[1][1] = 0; S[1][2] = -x[0];
    S[2][0] = -x[1]; S[2][1] = x[0]; S[2][2] = 0;
}

static void bk_apply(const double T[12], const double X[3], double x[3])
{
    for (int i = 0; i < 3; ++i) x[i] = T[4 * i] * X[0] + T[4 * i + 1] * X[1] + T[4 * i + 2] * X[2] + T[4 * i + 3];
}

/* A B for 3x4 similarity matrices (out may not alias). */
static void bk_mul(const double A[12], const double B[12], double out[12])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[4 * i + k] * B[4 * k + j];
            out[4 * i + j] = s + (j == 3 ? A[4 * i + 3] : 0.0);
        }
}

/* [sR | t]^-1 = [R^T / s | -R^T t / s]; s from the determinant's cube root. */
static void bk_inv(const double T[12], double out[12])
{
    double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                 T[2] * (T[4] * T[9] - T[5] * T[8]);
    double s = cbrt(det);
    double s2 = s * s;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[4 * i + j] = T[4 * j + i] / s2;  /* (sR)^T / s^2 = R^T / s */
    for (int i = 0; i < 3; ++i) {
        double v = 0.0;
        for (int k = 0; k < 3; ++k) v += out[4 * i + k] * T[4 * k + 3];
        out[4 * i + 3] = -v;
    }
}

/* Ad(T) as a 7x7 row-major matrix. */
static void bk_adjoint(const double T[12], double A[49])
{
    double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                 T[2] * (T[4] * T[9] - T[5] * T[8]);
    double s = cbrt(det);
    double R[3][3], t[3] = {T[3], T[7], T[11]}, S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = T[4 * i + j] / s;
    bk_skew(t, S);
    memset(A, 0, 49 * sizeof(double));
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double tr = 0.0;
            for (int k = 0; k < 3; ++k) tr += S[i][k] * R[k][j];
            A[7 * i + j] = s * R[i][j];
            A[7 * i + 3 + j] = tr;
            A[7 * (3 + i) + 3 + j] = R[i][j];
        }
        A[7 * i + 6] = -t[i];
    }
    A[7 * 6 + 6] = 1.0;
}

static double bk_huber_weight(double a, double width) { return a <= width ? 1.0 : width / a; }
static double bk_huber_cost(double a, double width) { return a <= width ? 0.5 * a * a : width * (a - 0.5 * width); }

/*
 * Residuals r[4] and their Jacobians w.r.t. left perturbations of the two
 * world poses, Ji[28] and Jj[28] (4x7 row-major), for one match: Xj_n is the
 * point of frame j at pixel n, Xi_m the point of frame i at its match m.
 * Returns 0 (and leaves the outputs) if a point is at the origin.
 */
int oracle_backend_residual(const double Ti[12], const double Tj[12], const double Xj_n[3], const double Xi_m[3],
                            double r[4], double Ji[28], double Jj[28])
{
    double Tii[12], Tij[12], A[49];
    bk_inv(Ti, Tii);
    bk_mul(Tii, Tj, Tij);
    bk_adjoint(Tii, A);
    double x[3];
    bk_apply(Tij, Xj_n, x);
    double d = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double dy = sqrt(Xi_m[0] * Xi_m[0] + Xi_m[1] * Xi_m[1] + Xi_m[2] * Xi_m[2]);
    if (!(d > 0.0) || !(dy > 0.0) || !isfinite(d) || !isfinite(dy)) return 0;
    double u[3] = {x[0] / d, x[1] / d, x[2] / d};
    double S[3][3], J[4][7];
    bk_skew(x, S);
    for (int a = 0; a < 3; ++a) {
        r[a] = u[a] - Xi_m[a] / dy;
        for (int b = 0; b < 3; ++b) {
            J[a][b] = ((a == b ? 1.0 : 0.0) - u[a] * u[b]) / d;
            J[a][3 + b] = -S[a][b] / d;
        }
        J[a][6] = 0.0;
    }
    r[3] = d - dy;
    for (int b = 0; b < 3; ++b) { J[3][b] = u[b]; J[3][3 + b] = 0.0; }
    J[3][6] = d;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 7; ++b) {
            double s = 0.0;
            for (int k = 0; k < 7; ++k) s += J[a][k] * A[7 * k + b];
            Ji[7 * a + b] = -s;
            Jj[7 * a + b] = s;
        }
    return 1;
}

typedef struct {
    double *H;   /* 7N x 7N */
    double *g;   /* 7N */
    double cost;
    long count;
} bk_system;

static void bk_build(int N, long HW, const double *Xc, const double *Q, int E, const int32_t *ei, const int32_t *ej,
                     const int32_t *idx, const uint8_t *valid, double q_min, double sigma_ray, double sigma_dist,
                     double huber, const double *T_WC, bk_system *sys)
{
    const int n7 = 7 * N;
    memset(sys->H, 0, sizeof(double) * n7 * n7);
    memset(sys->g, 0, sizeof(double) * n7);
    sys->cost = 0.0;
    sys->count = 0;
    for (int e = 0; e < E; ++e) {
        const int i = ei[e], j = ej[e];
        for (long n = 0; n < HW; ++n) {
            const long k = (long)e * HW + n;
            if (!valid[k] || idx[k] < 0) continue;
            const long m = idx[k];
            double q = sqrt(Q[(long)i * HW + m] * Q[(long)j * HW + n]);
            if (!(q > q_min)) continue;
            double r[4], Ji[28], Jj[28];
            if (!oracle_backend_residual(T_WC + 12 * i, T_WC + 12 * j, Xc + 3 * ((long)j * HW + n),
                                         Xc + 3 * ((long)i * HW + m), r, Ji, Jj))
                continue;
            double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            double a_ray = rn * sqrt(q) / sigma_ray;
            double a_dist = fabs(r[3]) * sqrt(q) / sigma_dist;
            double w_ray = q / (sigma_ray * sigma_ray) * bk_huber_weight(a_ray, huber);
            double w_dist = q / (sigma_dist * sigma_dist) * bk_huber_weight(a_dist, huber);
            double w[4] = {w_ray, w_ray, w_ray, w_dist};
            const double *Jb[2] = {Ji, Jj};
            const int blk[2] = {i, j};
            for (int p = 0; p < 2; ++p) {
                for (int a = 0; a < 7; ++a) {
                    double gg = 0.0;
                    for (int row = 0; row < 4; ++row) gg += Jb[p][7 * row + a] * w[row] * r[row];
                    sys->g[7 * blk[p] + a] += gg;
                    for (int c = 0; c < 2; ++c)
                        for (int b = 0; b < 7; ++b) {
                            double h = 0.0;
                            for (int row = 0; row < 4; ++row) h += Jb[p][7 * row + a] * w[row] * Jb[c][7 * row + b];
                            sys->H[(long)(7 * blk[p] + a) * n7 + 7 * blk[c] + b] += h;
                        }
                }
            }
            sys->cost += bk_huber_cost(a_ray, huber) + bk_huber_cost(a_dist, huber);
            sys->count += 1;
        }
    }
}

/* Dense Cholesky solve of the n x n SPD system M x = b (M overwritten); 0 if not PD. */
static int bk_cholesky_solve(int n, double *M, const double *b, double *x)
{
    for (int c = 0; c < n; ++c) {
        double d = M[(long)c * n + c];
        for (int k = 0; k < c; ++k) d -= M[(long)c * n + k] * M[(long)c * n + k];
        if (!(d > 0.0) || !isfinite(d)) return 0;
        d = sqrt(d);
        M[(long)c * n + c] = d;
        for (int r = c + 1; r < n; ++r) {
            double s = M[(long)r * n + c];
            for (int k = 0; k < c; ++k) s -= M[(long)r * n + k] * M[(long)c * n + k];
            M[(long)r * n + c] = s / d;
        }
    }
    for (int r = 0; r < n; ++r) {
        double s = b[r];
        for (int k = 0; k < r; ++k) s -= M[(long)r * n + k] * x[k];
        x[r] = s / M[(long)r * n + r];
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = x[r];
        for (int k = r + 1; k < n; ++k) s -= M[(long)k * n + r] * x[k];
        x[r] = s / M[(long)r * n + r];
    }
    return 1;
}

/*
 * oracle_backend_gn: Gauss-Newton over the keyframe poses T_WC (N*12,
 * updated in place; keyframe 0 is held).  Returns the number of applied
 * steps; *cost / *count: robust cost and matches used at the final poses;
 * *last_step: norm of the last applied step (0 if none).
 */
int oracle_backend_gn(int N, int H, int W, const double *Xc, const double *Q, int E, const int32_t *ei,
                      const int32_t *ej, const int32_t *idx, const uint8_t *valid, double q_min, double sigma_ray,
                      double sigma_dist, double huber, int iters, double step_tol, double *T_WC, double *cost,
                      long *count, double *last_step)
{
    const long HW = (long)H * W;
    const int n7 = 7 * N, nr = 7 * (N - 1);
    bk_system sys;
    sys.H = (double *)malloc(sizeof(double) * n7 * n7);
    sys.g = (double *)malloc(sizeof(double) * n7);
    double *M = (double *)malloc(sizeof(double) * (nr > 0 ? nr * nr : 1));
    double *b = (double *)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    double *tau = (double *)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    int applied = 0;
    *last_step = 0.0;
    for (int it = 0; it < iters && nr > 0; ++it) {
        bk_build(N, HW, Xc, Q, E, ei, ej, idx, valid, q_min, sigma_ray, sigma_dist, huber, T_WC, &sys);
        for (int r = 0; r < nr; ++r) {
            b[r] = -sys.g[7 + r];
            for (int c = 0; c < nr; ++c) M[(long)r * nr + c] = sys.H[(long)(7 + r) * n7 + 7 + c];
        }
        if (!bk_cholesky_solve(nr, M, b, tau)) break;
        double nrm = 0.0;
        for (int k = 1; k < N; ++k) {
            double E7[12], Tn[12];
            oracle_sim3_exp(tau + 7 * (k - 1), E7);
            bk_mul(E7, T_WC + 12 * k, Tn);
            memcpy(T_WC + 12 * k, Tn, sizeof Tn);
        }
        for (int r = 0; r < nr; ++r) nrm += tau[r] * tau[r];
        *last_step = sqrt(nrm);
        ++applied;
        if (*last_step < step_tol) break;
    }
    bk_build(N, HW, Xc, Q, E, ei, ej, idx, valid, q_min, sigma_ray, sigma_dist, huber, T_WC, &sys);
    *cost = sys.cost;
    *count = sys.count;
    free(sys.H); free(sys.g); free(M); free(b); free(tau);
    return applied;
}
