/*
 * FP64 CPU oracle for iterative projective pointmap matching
 * (MASt3R-SLAM, Murai, Dexheimer and Davison, CVPR 2025, arXiv 2412.12392).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the matcher computes.  It is used by the tests, by the
 * package's smoke check and by the CPU-baseline leg of the benchmark.  It shares
 * no code, header or constant with the HIP library and must never be linked
 * into it or called from the product path.
 *
 * Everything is computed in double precision from double inputs.  One query
 * pixel at a time, in the order the paper describes:
 *
 *   ray image         Sec. 3.1 (psi normalises a pointmap to unit rays) and
 *                     Fig. 2 (the reference pointmap is normalised first to give
 *                     a smooth pixel-to-ray map)
 *   ray error         Sec. 3.2, Eq. 2: p* = argmin_p |psi([X^i_i]_p) - psi(x)|^2
 *   angle             Sec. 3.2, Eq. 3: |psi1 - psi2|^2 = 2 (1 - cos theta)
 *   solver            Sec. 3.2: analytical Jacobians, Levenberg-Marquardt,
 *                     about 10 iterations, identity or given initialisation
 *   outlier gate      Sec. 3.2: invalidate matches far apart in 3D
 *   feature refine    Sec. 3.2: move to the best descriptor similarity in a
 *                     local window around the geometric match
 *   match confidence  Sec. 3.3: q = sqrt(Q^i_i[m] Q^j_i[n]), gated at q_min
 *   normalisation Jacobian  Supp. A, Eq. norm_jac: d psi / d x = (I - x x^T / d^2) / d
 *
 * Readings where the paper is silent (they are listed with reasons in the
 * design notes of the repository):
 *   pixel (x, y) = (column, row), pixel centres at integers, domain
 *     [0, W-1] x [0, H-1]; every iterate is clamped to it, and a coordinate
 *     sitting on its bound whose step points outward is held while the other
 *     coordinate takes its own 1-D damped step;
 *   the ray image is sampled bilinearly (cell origin x0 = min(floor(x), W-2))
 *     and the sample renormalised to unit length;
 *   the LM Jacobian uses bilinear samples of central-difference gradient
 *     images of the ray image (one-sided at the border);
 *   K iterations exactly, no early exit; damping lambda I, x10 on a rejected
 *     step, /10 on an accepted one, acceptance on strictly lower cost;
 *   theta = 2 asin(min(1, sqrt(c) / 2)), which is Eq. 3 solved for theta;
 *   refine: radius r around round-half-up of p*, raw dot products, first
 *     strict maximum in row-major window order; coarse-to-fine as `levels`
 *     levels of spacing 2^(levels-1), ..., 2, 1, each around the previous
 *     level's best (one level is the plain window);
 *   a reference pixel whose point is non-finite or zero has a zero ray; a
 *     sample whose interpolated ray is zero has infinite cost and a zero
 *     Jacobian; a query point that is non-finite or zero, or a non-finite
 *     initial pixel, gives an invalid match (idx -1, theta +inf, p = the
 *     clamped initial pixel, or 0 if that is non-finite).
 *
 * Backward (no counterpart in the paper): the implicit adjoint of the
 * converged match.  At p* the residual e(p*) = psi_hat(p*) - psi(x) vanishes,
 * so the derivative of p* by any input theta is -(Je^T Je)^-1 Je^T de/dtheta,
 * with Je the exact derivative of
 * the bilinear ray sampler (not the gradient-image Jacobian, which is only a
 * search direction and does not move the root).  A coordinate of p* held on
 * the image bound does not move; the other coordinate's derivative then comes
 * from its own 1-D system.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Ray image and its gradient images (Sec. 3.1, Fig. 2).               */
/* ------------------------------------------------------------------ */

static int finite3(const double *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

/* R[m] = X[m] / |X[m]|, zero for a non-finite or zero point. */
static void ray_image(int H, int W, const double *X, double *R)
{
    for (long m = 0; m < (long)H * W; ++m) {
        const double *x = X + 3 * m;
        double n = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (finite3(x) && n > 0.0 && isfinite(n)) {
            R[3 * m + 0] = x[0] / n;
            R[3 * m + 1] = x[1] / n;
            R[3 * m + 2] = x[2] / n;
        } else {
            R[3 * m + 0] = R[3 * m + 1] = R[3 * m + 2] = 0.0;
        }
    }
}

/* Gx[y,x] = (R[y,x+] - R[y,x-]) / (x+ - x-), x+- = clamp(x +- 1); Gy likewise. */
static void gradient_images(int H, int W, const double *R, double *Gx, double *Gy)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int xm = x > 0 ? x - 1 : 0, xp = x < W - 1 ? x + 1 : W - 1;
            int ym = y > 0 ? y - 1 : 0, yp = y < H - 1 ? y + 1 : H - 1;
            long m = (long)y * W + x;
            for (int c = 0; c < 3; ++c) {
                Gx[3 * m + c] = (R[3 * ((long)y * W + xp) + c] - R[3 * ((long)y * W + xm) + c]) / (double)(xp - xm);
                Gy[3 * m + c] = (R[3 * ((long)yp * W + x) + c] - R[3 * ((long)ym * W + x) + c]) / (double)(yp - ym);
            }
        }
    }
}

typedef struct {
    int H, W;
    const double *R, *Gx, *Gy;
} ray_map;

/* Bilinear cell and weights of pixel p; requires H, W >= 2 and p in the domain. */
typedef struct { long m00, m10, m01, m11; double a, b; } cell;

static cell cell_of(int H, int W, double px, double py)
{
    cell c;
    int x0 = (int)floor(px), y0 = (int)floor(py);
    if (x0 > W - 2) x0 = W - 2;
    if (y0 > H - 2) y0 = H - 2;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    c.a = px - x0;
    c.b = py - y0;
    c.m00 = (long)y0 * W + x0;
    c.m10 = c.m00 + 1;
    c.m01 = c.m00 + W;
    c.m11 = c.m01 + 1;
    return c;
}

static void bilerp3(const double *I, const cell *c, double out[3])
{
    double w00 = (1 - c->a) * (1 - c->b), w10 = c->a * (1 - c->b);
    double w01 = (1 - c->a) * c->b, w11 = c->a * c->b;
    for (int k = 0; k < 3; ++k)
        out[k] = w00 * I[3 * c->m00 + k] + w10 * I[3 * c->m10 + k] + w01 * I[3 * c->m01 + k] + w11 * I[3 * c->m11 + k];
}

/* One evaluation of the ray error of Eq. 2 at pixel p for target ray t. */
typedef struct { double c; double e[3]; double J[3][2]; } sample_t;

static void sample_ray_error(const ray_map *rm, double px, double py, const double t[3], sample_t *s)
{
    cell cl = cell_of(rm->H, rm->W, px, py);
    double r[3], gx[3], gy[3];
    bilerp3(rm->R, &cl, r);
    bilerp3(rm->Gx, &cl, gx);
    bilerp3(rm->Gy, &cl, gy);
    double n2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    if (!(n2 > 0.0) || !isfinite(n2)) {
        s->c = INFINITY;
        memset(s->e, 0, sizeof s->e);
        memset(s->J, 0, sizeof s->J);
        return;
    }
    double n = sqrt(n2);
    double psi[3] = {r[0] / n, r[1] / n, r[2] / n};
    /* d psi_hat / d p = (I - psi psi^T) [gx gy] / |r|  (Supp. A, Eq. norm_jac). */
    double pgx = psi[0] * gx[0] + psi[1] * gx[1] + psi[2] * gx[2];
    double pgy = psi[0] * gy[0] + psi[1] * gy[1] + psi[2] * gy[2];
    double c = 0.0;
    for (int k = 0; k < 3; ++k) {
        s->J[k][0] = (gx[k] - psi[k] * pgx) / n;
        s->J[k][1] = (gy[k] - psi[k] * pgy) / n;
        s->e[k] = psi[k] - t[k];
        c += s->e[k] * s->e[k];
    }
    s->c = c;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------ */
/* Forward: LM projection, residual angle, window refine, gates.       */
/* ------------------------------------------------------------------ */

typedef struct {
    int H, W, D, K, r, levels;
    double lambda0, conf_min, max_theta, max_dist;
    const double *Xii, *Xji, *Dii, *Dji, *Qii, *Qji, *p_init;
    ray_map rm;
    double *p, *theta, *xhat, *gap;
    int32_t *idx;
    uint8_t *valid;
} fwd_ctx;

static void match_one(const fwd_ctx *C, long n)
{
    const int H = C->H, W = C->W;
    const double *x = C->Xji + 3 * n;
    double px0, py0;
    int bad = 0;
    if (C->p_init) {
        px0 = C->p_init[2 * n + 0];
        py0 = C->p_init[2 * n + 1];
        if (!isfinite(px0) || !isfinite(py0)) { bad = 1; px0 = py0 = 0.0; }
    } else {
        px0 = (double)(n % W);
        py0 = (double)(n / W);
    }
    double px = clampd(px0, 0.0, W - 1.0), py = clampd(py0, 0.0, H - 1.0);

    double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    if (!finite3(x) || !(xn > 0.0) || !isfinite(xn)) bad = 1;

    C->p[2 * n + 0] = px;
    C->p[2 * n + 1] = py;
    if (C->xhat) { C->xhat[3 * n] = C->xhat[3 * n + 1] = C->xhat[3 * n + 2] = NAN; }
    if (C->gap) C->gap[n] = NAN;
    if (bad) {
        C->idx[n] = -1;
        C->valid[n] = 0;
        if (C->theta) C->theta[n] = INFINITY;
        return;
    }

    /* Target ray psi(x) (Sec. 3.1). */
    double t[3] = {x[0] / xn, x[1] / xn, x[2] / xn};

    /* Levenberg-Marquardt on Eq. 2 (Sec. 3.2). */
    sample_t cur, nxt;
    sample_ray_error(&C->rm, px, py, t, &cur);
    double lambda = C->lambda0;
    for (int it = 0; it < C->K; ++it) {
        double a00 = 0, a01 = 0, a11 = 0, g0 = 0, g1 = 0;
        for (int k = 0; k < 3; ++k) {
            a00 += cur.J[k][0] * cur.J[k][0];
            a01 += cur.J[k][0] * cur.J[k][1];
            a11 += cur.J[k][1] * cur.J[k][1];
            g0 += cur.J[k][0] * cur.e[k];
            g1 += cur.J[k][1] * cur.e[k];
        }
        a00 += lambda;
        a11 += lambda;
        double det = a00 * a11 - a01 * a01;
        double dx = -(a11 * g0 - a01 * g1) / det;
        double dy = -(a00 * g1 - a01 * g0) / det;
        if (!isfinite(dx) || !isfinite(dy)) { lambda *= 10.0; continue; }
        /* Bounds: a coordinate on its bound whose step points out of the image
           is held; the other coordinate takes its own 1-D damped step. */
        int hold_x = (px <= 0.0 && dx < 0.0) || (px >= W - 1.0 && dx > 0.0);
        int hold_y = (py <= 0.0 && dy < 0.0) || (py >= H - 1.0 && dy > 0.0);
        if (hold_x && hold_y) { dx = 0.0; dy = 0.0; }
        else if (hold_x) { dx = 0.0; dy = -g1 / a11; }
        else if (hold_y) { dy = 0.0; dx = -g0 / a00; }
        double qx = clampd(px + dx, 0.0, W - 1.0), qy = clampd(py + dy, 0.0, H - 1.0);
        sample_ray_error(&C->rm, qx, qy, t, &nxt);
        if (nxt.c < cur.c) {
            px = qx; py = qy; cur = nxt;
            lambda /= 10.0;
        } else {
            lambda *= 10.0;
        }
    }
    C->p[2 * n + 0] = px;
    C->p[2 * n + 1] = py;

    /* Residual angle from Eq. 3: c = |e|^2 = 2 (1 - cos th) = 4 sin^2(th / 2). */
    double th = 2.0 * asin(fmin(1.0, sqrt(cur.c) / 2.0));
    if (C->theta) C->theta[n] = th;

    if (C->xhat) {
        cell cl = cell_of(H, W, px, py);
        bilerp3(C->Xii, &cl, C->xhat + 3 * n);
    }

    /* Feature refine (Sec. 3.2): coarse-to-fine search for the best raw
       descriptor dot product.  Level l, from levels-1 down to 0, scans the
       (2r+1)^2 grid of spacing 2^l around the current centre (first strict
       maximum in row-major order) and moves the centre there; the first
       centre is the match rounded half up.  One level is the plain window. */
    int mx0 = (int)floor(px + 0.5), my0 = (int)floor(py + 0.5);
    const double *dq = C->Dji + (long)C->D * n;
    double best = -INFINITY, second = -INFINITY;
    long best_m = -1;
    for (int lev = C->levels - 1; lev >= 0; --lev) {
        const int sp = 1 << lev;
        long lev_m = -1;
        best = -INFINITY;
        second = -INFINITY;
        for (int dy = -C->r; dy <= C->r; ++dy) {
            int my = my0 + sp * dy;
            if (my < 0 || my >= H) continue;
            for (int dx = -C->r; dx <= C->r; ++dx) {
                int mx = mx0 + sp * dx;
                if (mx < 0 || mx >= W) continue;
                long m = (long)my * W + mx;
                const double *dr = C->Dii + (long)C->D * m;
                double s = 0.0;
                for (int k = 0; k < C->D; ++k) s += dq[k] * dr[k];
                if (s > best) { second = best; best = s; lev_m = m; }
                else if (s > second) second = s;
            }
        }
        if (lev_m < 0) break;
        best_m = lev_m;
        mx0 = (int)(lev_m % W);
        my0 = (int)(lev_m / W);
    }
    C->idx[n] = (int32_t)best_m;
    if (C->gap) C->gap[n] = best - second;

    /* Gates: residual angle, match confidence (Sec. 3.3), 3D distance (Sec. 3.2). */
    int ok = best_m >= 0 && th <= C->max_theta;
    if (ok && C->Qii && C->Qji) ok = sqrt(C->Qii[best_m] * C->Qji[n]) >= C->conf_min;
    if (ok && C->max_dist < INFINITY) {
        const double *xr = C->Xii + 3 * best_m;
        double d0 = xr[0] - x[0], d1 = xr[1] - x[1], d2 = xr[2] - x[2];
        ok = sqrt(d0 * d0 + d1 * d1 + d2 * d2) <= C->max_dist;
    }
    C->valid[n] = (uint8_t)(ok ? 1 : 0);
}

/*
 * oracle_match_fwd: match every pixel of Xji against frame i.
 *   H, W >= 2, D >= 1; arrays row-major, pixel m = y * W + x:
 *   Xii, Xji [H*W*3]; Dii, Dji [H*W*D]; Qii, Qji [H*W] or both NULL;
 *   p_init [H*W*2] as (x, y) or NULL for the identity initialisation.
 * levels >= 1: coarse-to-fine refine levels (1 = single window).
 * Outputs: p [H*W*2] (continuous p* before refine), idx [H*W] (refined
 *   linear index, -1 if none), valid [H*W]; optional (may be NULL): theta
 *   [H*W], xhat [H*W*3] (bilinear X^i_i at p*), gap [H*W] (best minus
 *   second-best window score of the last level, +inf if there is one
 *   candidate).
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad sizes.
 */
int oracle_match_fwd(int H, int W, int D,
                     const double *Xii, const double *Xji, const double *Dii, const double *Dji,
                     const double *Qii, const double *Qji, const double *p_init,
                     int K, double lambda0, int r, int levels, double conf_min, double max_theta, double max_dist,
                     double *p, int32_t *idx, uint8_t *valid, double *theta, double *xhat, double *gap,
                     int nthreads)
{
    if (H < 2 || W < 2 || D < 1 || K < 0 || r < 0 || levels < 1 || levels > 16) return -1;
    long N = (long)H * W;
    double *R = malloc(sizeof(double) * 3 * N), *Gx = malloc(sizeof(double) * 3 * N),
           *Gy = malloc(sizeof(double) * 3 * N);
    if (!R || !Gx || !Gy) { free(R); free(Gx); free(Gy); return -2; }
    ray_image(H, W, Xii, R);
    gradient_images(H, W, R, Gx, Gy);
    fwd_ctx C = {H, W, D, K, r, levels, lambda0, conf_min, max_theta, max_dist,
                 Xii, Xji, Dii, Dji, (Qii && Qji) ? Qii : NULL, (Qii && Qji) ? Qji : NULL, p_init,
                 {H, W, R, Gx, Gy}, p, theta, xhat, gap, idx, valid};
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
#endif
    for (long n = 0; n < N; ++n) match_one(&C, n);
    (void)nthreads;
    free(R); free(Gx); free(Gy);
    return 0;
}

/* Number of threads the OpenMP runtime would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * oracle_cost_grid: the ray error c(p) of Eq. 2 for one target point x at
 * npts pixels (px[k], py[k]) (clamped to the domain).  For brute-force scans.
 */
int oracle_cost_grid(int H, int W, const double *Xii, const double *x, long npts,
                     const double *px, const double *py, double *cost)
{
    if (H < 2 || W < 2) return -1;
    long N = (long)H * W;
    double *R = malloc(sizeof(double) * 3 * N), *Gx = malloc(sizeof(double) * 3 * N),
           *Gy = malloc(sizeof(double) * 3 * N);
    if (!R || !Gx || !Gy) { free(R); free(Gx); free(Gy); return -2; }
    ray_image(H, W, Xii, R);
    gradient_images(H, W, R, Gx, Gy);
    ray_map rm = {H, W, R, Gx, Gy};
    double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double t[3] = {x[0] / xn, x[1] / xn, x[2] / xn};
    for (long k = 0; k < npts; ++k) {
        sample_t s;
        sample_ray_error(&rm, clampd(px[k], 0.0, W - 1.0), clampd(py[k], 0.0, H - 1.0), t, &s);
        cost[k] = s.c;
    }
    free(R); free(Gx); free(Gy);
    return 0;
}

/* oracle_ray_images: the ray image R and its gradient images Gx, Gy, [H*W*3] each. */
int oracle_ray_images(int H, int W, const double *Xii, double *R, double *Gx, double *Gy)
{
    if (H < 2 || W < 2) return -1;
    ray_image(H, W, Xii, R);
    gradient_images(H, W, R, Gx, Gy);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Backward: implicit adjoint of the converged match.                  */
/* ------------------------------------------------------------------ */

/* N(X) v = (I - u u^T) v / |X| with u = X / |X|  (Supp. A, Eq. norm_jac). */
static void norm_jac_apply(const double *X, const double v[3], double out[3])
{
    double n = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    double u[3] = {X[0] / n, X[1] / n, X[2] / n};
    double uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    for (int k = 0; k < 3; ++k) out[k] = (v[k] - u[k] * uv) / n;
}

/*
 * oracle_match_bwd: given the forward's p and valid, and upstream gradients
 * grad_p [H*W*2] and grad_xhat [H*W*3] (may be NULL), write dL/dXii and
 * dL/dXji [H*W*3] each (overwritten) for the path through the match p* and
 * the sampled point xhat = bilinear(Xii, p*).  Invalid queries contribute 0,
 * as do queries whose 2x2 system is singular.
 */
int oracle_match_bwd(int H, int W, const double *Xii, const double *Xji,
                     const double *p, const uint8_t *valid,
                     const double *grad_p, const double *grad_xhat,
                     double *dXii, double *dXji)
{
    if (H < 2 || W < 2) return -1;
    long N = (long)H * W;
    double *R = malloc(sizeof(double) * 3 * N);
    if (!R) return -2;
    ray_image(H, W, Xii, R);
    memset(dXii, 0, sizeof(double) * 3 * N);
    memset(dXji, 0, sizeof(double) * 3 * N);
    for (long n = 0; n < N; ++n) {
        if (!valid[n]) continue;
        cell cl = cell_of(H, W, p[2 * n], p[2 * n + 1]);
        double a = cl.a, b = cl.b;
        const double *R00 = R + 3 * cl.m00, *R10 = R + 3 * cl.m10, *R01 = R + 3 * cl.m01, *R11 = R + 3 * cl.m11;
        double r[3];
        bilerp3(R, &cl, r);
        /* Exact derivatives of the bilinear ray sample r(p). */
        double drx[3], dry[3];
        for (int k = 0; k < 3; ++k) {
            drx[k] = (1 - b) * (R10[k] - R00[k]) + b * (R11[k] - R01[k]);
            dry[k] = (1 - a) * (R01[k] - R00[k]) + a * (R11[k] - R10[k]);
        }
        double Je[3][2], col[3];
        norm_jac_apply(r, drx, col);
        for (int k = 0; k < 3; ++k) Je[k][0] = col[k];
        norm_jac_apply(r, dry, col);
        for (int k = 0; k < 3; ++k) Je[k][1] = col[k];

        double w[4] = {(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b};
        long cm[4] = {cl.m00, cl.m10, cl.m01, cl.m11};

        double gp0 = grad_p ? grad_p[2 * n] : 0.0, gp1 = grad_p ? grad_p[2 * n + 1] : 0.0;
        if (grad_xhat) {
            const double *gx = grad_xhat + 3 * n;
            const double *X00 = Xii + 3 * cl.m00, *X10 = Xii + 3 * cl.m10, *X01 = Xii + 3 * cl.m01, *X11 = Xii + 3 * cl.m11;
            for (int k = 0; k < 3; ++k) {
                double dxx = (1 - b) * (X10[k] - X00[k]) + b * (X11[k] - X01[k]);
                double dxy = (1 - a) * (X01[k] - X00[k]) + a * (X11[k] - X10[k]);
                gp0 += dxx * gx[k];
                gp1 += dxy * gx[k];
            }
            /* Direct dependence of xhat on the four corner points. */
            for (int c = 0; c < 4; ++c)
                for (int k = 0; k < 3; ++k) dXii[3 * cm[c] + k] += w[c] * gx[k];
        }
        /* mu = (Je^T Je)^-1 g_p, v = Je mu.  A coordinate of p* on its bound
           is held by the forward, so it does not move: it drops out and the
           other coordinate is solved alone (both held: p* does not move). */
        double a00 = 0, a01 = 0, a11 = 0;
        for (int k = 0; k < 3; ++k) {
            a00 += Je[k][0] * Je[k][0];
            a01 += Je[k][0] * Je[k][1];
            a11 += Je[k][1] * Je[k][1];
        }
        int held_x = p[2 * n] <= 0.0 || p[2 * n] >= W - 1.0;
        int held_y = p[2 * n + 1] <= 0.0 || p[2 * n + 1] >= H - 1.0;
        double mu0 = 0.0, mu1 = 0.0;
        if (held_x && held_y) {
            /* nothing moves */
        } else if (held_x) {
            if (!(a11 > 0.0)) continue;
            mu1 = gp1 / a11;
        } else if (held_y) {
            if (!(a00 > 0.0)) continue;
            mu0 = gp0 / a00;
        } else {
            double det = a00 * a11 - a01 * a01;
            if (!(det > 0.0) || !isfinite(det)) continue;
            mu0 = (a11 * gp0 - a01 * gp1) / det;
            mu1 = (a00 * gp1 - a01 * gp0) / det;
        }
        double v[3];
        for (int k = 0; k < 3; ++k) v[k] = Je[k][0] * mu0 + Je[k][1] * mu1;

        /* e = psi_hat(p; X^i_i) - psi(x):  dL/dx = +N(x) v,
           dL/dX^i_i[c] = -w_c N(X^i_i[c]) N(r) v = -(w_c / |r|) N(X^i_i[c]) v. */
        double out[3];
        norm_jac_apply(Xji + 3 * n, v, out);
        for (int k = 0; k < 3; ++k) dXji[3 * n + k] = out[k];
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int c = 0; c < 4; ++c) {
            /* A corner with zero weight, or whose point has no ray, has no
               derivative through the ray image. */
            const double *Rc = R + 3 * cm[c];
            if (w[c] == 0.0 || (Rc[0] == 0.0 && Rc[1] == 0.0 && Rc[2] == 0.0)) continue;
            norm_jac_apply(Xii + 3 * cm[c], v, out);
            for (int k = 0; k < 3; ++k) dXii[3 * cm[c] + k] -= (w[c] / rn) * out[k];
        }
    }
    free(R);
    return 0;
}
