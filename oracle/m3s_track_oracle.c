/*
 * FP64 CPU oracle for the tracking pose solve of MASt3R-SLAM (Sec. 3.3).
 *
 * TEST INFRASTRUCTURE ONLY (see m3s_oracle.c): shares no code with the HIP
 * library and is never linked into it.
 *
 * Given the canonical keyframe pointmap Xk (the measured points, H*W*3), the
 * current frame's pointmap Xf (H*W*3), the matches idx[n] (keyframe pixel n
 * -> frame pixel m, from the matcher) with their valid flags, and the
 * confidences Qf[m], Qk[n], it refines the Sim(3) pose T_kf = [sR | t] that
 * maps frame points into the keyframe, by Gauss-Newton in an iteratively
 * reweighted least-squares loop (Eq. gauss_newton):
 *
 *   for every valid match with q = sqrt(Qf[m] Qk[n]) > q_min (Sec. 3.3,
 *   match confidence and w(q, sigma^2)):
 *     x    = T Xf[m]
 *     r_ray  = psi(x) - psi(Xk[n])          ray residual (Eq. track_ray,
 *                                            transformed minus measured as in
 *                                            Supp. A)
 *     r_dist = |x| - |Xk[n]|                 distance residual (Sec. 3.3, the
 *                                            small-weight distance term)
 *     J_ray  = [N(x), -[x]_x / |x|, 0]       Supp. A, Eq. norm_jac and the ray
 *                                            Jacobian w.r.t. the pose
 *     J_dist = [x^T / |x|, 0, |x|]           Supp. A, Eq. dist_jac
 *     weights: q / sigma^2 times the Huber weight of the whitened residual
 *   solve (sum J^T W J) tau = -(sum J^T W r) (7x7), T <- Exp(tau) o T (Eq. 1,
 *   left plus on Sim(3)), for a fixed number of iterations.
 *
 * Tangent order tau = (v, omega, sigma): translation, rotation, log-scale,
 * matching the point Jacobian [I, -[x]_x, x] of Supp. A (Eq. point_jac).
 * Readings where the paper is silent: the Huber norm acts on the whitened
 * block norm |r| sqrt(q) / sigma with width `huber`; w(q, sigma^2) = sigma^2/q
 * divides the squared residual; fixed iteration count; a 7x7 system solved by
 * Cholesky, the step skipped if it is not positive definite.
 *
 * Pose layout: double T[12] = row-major 3x4 [sR | t].
 *
 * The file also holds the canonical pointmap fusion that follows the pose
 * solve (Eq. 8), oracle_fuse.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    double H[7][7];
    double g[7];
    double cost;
    long count;
} normal_eq;

static void skew(const double x[3], double S[3][3])
{
    S[0][0] = 0; S[0][1] = -x[2]; S[0][2] = x[1];
    S[1][0] = x[2]; S[1][1] = 0; S[1][2] = -x[0];
    S[2][0] = -x[1]; S[2][1] = x[0]; S[2][2] = 0;
}

/* Huber weight of a whitened norm a: 1 inside the width, width / a outside. */
static double huber_weight(double a, double width) { return a <= width ? 1.0 : width / a; }

/* Huber cost of a whitened norm a (0.5 a^2 inside, width (a - width/2) outside). */
static double huber_cost(double a, double width) { return a <= width ? 0.5 * a * a : width * (a - 0.5 * width); }

static void apply_pose(const double T[12], const double X[3], double x[3])
{
    for (int i = 0; i < 3; ++i) x[i] = T[4 * i] * X[0] + T[4 * i + 1] * X[1] + T[4 * i + 2] * X[2] + T[4 * i + 3];
}

/* Accumulate the weighted normal equations of all matches at pose T. */
static void build_normal_equations(long N, const double *Xk, const double *Xf, const int32_t *idx,
                                   const uint8_t *valid, const double *Qf, const double *Qk,
                                   const double T[12], double q_min, double sigma_ray, double sigma_dist,
                                   double huber, normal_eq *ne)
{
    memset(ne, 0, sizeof *ne);
    for (long n = 0; n < N; ++n) {
        if (!valid[n] || idx[n] < 0) continue;
        long m = idx[n];
        double q = sqrt(Qf[m] * Qk[n]);
        if (!(q > q_min)) continue;
        const double *Y = Xk + 3 * n;
        double x[3];
        apply_pose(T, Xf + 3 * m, x);
        double d = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double dy = sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]);
        if (!(d > 0.0) || !(dy > 0.0) || !isfinite(d) || !isfinite(dy)) continue;
        double u[3] = {x[0] / d, x[1] / d, x[2] / d};
        double r[3] = {u[0] - Y[0] / dy, u[1] - Y[1] / dy, u[2] - Y[2] / dy};
        double rd = d - dy;

        /* J_ray = [N(x), -[x]_x / d, 0], N(x) = (I - u u^T) / d. */
        double J[4][7];
        double S[3][3];
        skew(x, S);
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                J[i][j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]) / d;
                J[i][3 + j] = -S[i][j] / d;
            }
            J[i][6] = 0.0;
        }
        /* J_dist = [x^T / d, 0, d]. */
        for (int j = 0; j < 3; ++j) { J[3][j] = u[j]; J[3][3 + j] = 0.0; }
        J[3][6] = d;

        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double a_ray = rn * sqrt(q) / sigma_ray;
        double a_dist = fabs(rd) * sqrt(q) / sigma_dist;
        double w_ray = q / (sigma_ray * sigma_ray) * huber_weight(a_ray, huber);
        double w_dist = q / (sigma_dist * sigma_dist) * huber_weight(a_dist, huber);
        double res[4] = {r[0], r[1], r[2], rd};
        double w[4] = {w_ray, w_ray, w_ray, w_dist};
        for (int a = 0; a < 7; ++a) {
            for (int b = 0; b < 7; ++b) {
                double h = 0.0;
                for (int k = 0; k < 4; ++k) h += J[k][a] * w[k] * J[k][b];
                ne->H[a][b] += h;
            }
            double gg = 0.0;
            for (int k = 0; k < 4; ++k) gg += J[k][a] * w[k] * res[k];
            ne->g[a] += gg;
        }
        ne->cost += huber_cost(a_ray, huber) + huber_cost(a_dist, huber);
        ne->count += 1;
    }
}

/* Solve H x = b (7x7, symmetric) by Cholesky; returns 0 if H is not positive definite. */
static int cholesky_solve7(double H[7][7], const double b[7], double x[7])
{
    double L[7][7];
    memset(L, 0, sizeof L);
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = H[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return 0;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[7];
    for (int i = 0; i < 7; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = 6; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 7; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return 1;
}

/*
 * Exp of sim(3) (Eq. 1): tau = (v, omega, sigma) -> [e^sigma R | V v] with
 * R = exp([omega]_x) (Rodrigues) and V = int_0^1 e^{sigma s} exp(s [omega]_x) ds
 * = a0 I + a1 [omega]_x + a2 [omega]_x^2.  Series forms near theta = 0 and
 * sigma = 0.
 */
void oracle_sim3_exp(const double tau[7], double T[12])
{
    const double *v = tau, *w = tau + 3;
    double sigma = tau[6];
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double S[3][3], S2[3][3];
    skew(w, S);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += S[i][k] * S[k][j];
            S2[i][j] = s;
        }
    double ka, kb; /* R = I + ka S + kb S^2 */
    if (th < 1e-4) { ka = 1.0 - th2 / 6.0; kb = 0.5 - th2 / 24.0; }
    else { ka = sin(th) / th; kb = (1.0 - cos(th)) / th2; }
    double es = exp(sigma);
    double a0, a1, a2;
    if (sigma == 0.0) a0 = 1.0;
    else a0 = expm1(sigma) / sigma;
    if (th < 1e-4) {
        /* Taylor in theta: int e^{sigma s} s ds and int e^{sigma s} s^2/2 ds,
           by their own series when sigma is small (the closed forms cancel). */
        double i1, i2, s2 = sigma * sigma;
        if (fabs(sigma) < 1e-3) {
            i1 = 0.5 + sigma / 3.0 + s2 / 8.0 + s2 * sigma / 30.0;
            i2 = 1.0 / 6.0 + sigma / 8.0 + s2 / 20.0 + s2 * sigma / 72.0;
        } else {
            i1 = (es * (sigma - 1.0) + 1.0) / (sigma * sigma);
            i2 = (es * (sigma * sigma - 2.0 * sigma + 2.0) - 2.0) / (2.0 * sigma * sigma * sigma);
        }
        a1 = i1;
        a2 = i2;
    } else {
        double den = sigma * sigma + th2;
        double is = (es * (sigma * sin(th) - th * cos(th)) + th) / den;   /* int e^{sigma s} sin(th s) ds */
        double ic = (es * (sigma * cos(th) + th * sin(th)) - sigma) / den; /* int e^{sigma s} cos(th s) ds */
        a1 = is / th;
        a2 = (a0 - ic) / th2;
    }
    for (int i = 0; i < 3; ++i) {
        double tv = 0.0;
        for (int j = 0; j < 3; ++j) {
            double R = (i == j ? 1.0 : 0.0) + ka * S[i][j] + kb * S2[i][j];
            double V = (i == j ? a0 : 0.0) + a1 * S[i][j] + a2 * S2[i][j];
            T[4 * i + j] = es * R;
            tv += V * v[j];
        }
        T[4 * i + 3] = tv;
    }
}

/* T <- A o T for 3x4 similarity matrices. */
static void compose(const double A[12], double T[12])
{
    double out[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[4 * i + k] * T[4 * k + j];
            if (j == 3) s += A[4 * i + 3];
            out[4 * i + j] = s;
        }
    }
    memcpy(T, out, sizeof out);
}

/*
 * oracle_track_pose: `iters` Gauss-Newton IRLS iterations from T (3x4,
 * updated in place).  Returns the number of iterations whose system was
 * solved; *cost receives the robust cost at the final pose and *count the
 * number of matches used there.  H_out / g_out (may be NULL) receive the
 * normal equations at the final pose (7x7 row-major, 7).
 */
int oracle_track_pose(int H, int W, const double *Xk, const double *Xf, const int32_t *idx, const uint8_t *valid,
                      const double *Qf, const double *Qk, double q_min, double sigma_ray, double sigma_dist,
                      double huber, int iters, double T[12], double *cost, long *count, double *H_out, double *g_out)
{
    long N = (long)H * W;
    int solved = 0;
    normal_eq ne;
    for (int it = 0; it < iters; ++it) {
        build_normal_equations(N, Xk, Xf, idx, valid, Qf, Qk, T, q_min, sigma_ray, sigma_dist, huber, &ne);
        double b[7], tau[7];
        for (int a = 0; a < 7; ++a) b[a] = -ne.g[a];
        if (!cholesky_solve7(ne.H, b, tau)) continue;
        double E[12];
        oracle_sim3_exp(tau, E);
        compose(E, T);
        ++solved;
    }
    build_normal_equations(N, Xk, Xf, idx, valid, Qf, Qk, T, q_min, sigma_ray, sigma_dist, huber, &ne);
    if (cost) *cost = ne.cost;
    if (count) *count = ne.count;
    if (H_out) for (int a = 0; a < 7; ++a) for (int b = 0; b < 7; ++b) H_out[7 * a + b] = ne.H[a][b];
    if (g_out) for (int a = 0; a < 7; ++a) g_out[a] = ne.g[a];
    return solved;
}

/*
 * oracle_track_residual: ray and distance residuals and Jacobians of one
 * match at pose T (for finite-difference pins): r[4], J[4*7] row-major.
 */
void oracle_track_residual(const double T[12], const double Xf_m[3], const double Xk_n[3], double r[4], double J[28])
{
    double x[3];
    apply_pose(T, Xf_m, x);
    double d = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double dy = sqrt(Xk_n[0] * Xk_n[0] + Xk_n[1] * Xk_n[1] + Xk_n[2] * Xk_n[2]);
    double u[3] = {x[0] / d, x[1] / d, x[2] / d};
    double S[3][3];
    skew(x, S);
    for (int i = 0; i < 3; ++i) {
        r[i] = u[i] - Xk_n[i] / dy;
        for (int j = 0; j < 3; ++j) {
            J[7 * i + j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]) / d;
            J[7 * i + 3 + j] = -S[i][j] / d;
        }
        J[7 * i + 6] = 0.0;
    }
    r[3] = d - dy;
    for (int j = 0; j < 3; ++j) { J[21 + j] = u[j]; J[24 + j] = 0.0; }
    J[27] = d;
}

/*
 * oracle_fuse: the canonical pointmap update after tracking (Sec. 3.3, Eq. 8),
 * per keyframe pixel n:
 *   Xc[n] <- (Cc[n] Xc[n] + C[n] (T X[n])) / (Cc[n] + C[n]),  Cc[n] <- Cc[n] + C[n]
 * where X is the frame's prediction of the keyframe's pointmap (X^k_f) and T
 * the solved pose T_kf.  Reading where the paper is silent: a pixel whose
 * summed confidence is not positive keeps its point (only Cc is updated).
 * Xc (N*3) and Cc (N) are updated in place.
 */
void oracle_fuse(long N, const double T[12], double *Xc, double *Cc, const double *X, const double *C)
{
    for (long n = 0; n < N; ++n) {
        double x[3];
        apply_pose(T, X + 3 * n, x);
        double c_old = Cc[n], c_new = C[n];
        double c_sum = c_old + c_new;
        if (c_sum > 0.0) {
            for (int k = 0; k < 3; ++k) Xc[3 * n + k] = (c_old * Xc[3 * n + k] + c_new * x[k]) / c_sum;
        }
        Cc[n] = c_sum;
    }
}
