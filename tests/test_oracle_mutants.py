"""Planted mistakes in the oracle must fail at least one pin.

Each mutant is a textual edit of ``oracle/m3s_oracle.c`` (a dropped term, a
wrong sign or index, a transposed operand, a wrong tie-break...).  The edited
copy is compiled to a temporary library on the CPU and the pin battery of
``pins.py`` runs against it in a child process (so a mutant that crashes also
counts as caught).  A mutant that survives every pin means the pins would not
notice that mistake in the oracle.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "gradient_not_divided": [("/ (double)(xp - xm);", ";")],
    "gy_uses_x_neighbours": [("(R[3 * ((long)yp * W + x) + c] - R[3 * ((long)ym * W + x) + c])",
                              "(R[3 * ((long)y * W + xp) + c] - R[3 * ((long)y * W + xm) + c])")],
    "step_sign": [("double dx = -(a11 * g0 - a01 * g1) / det;", "double dx = (a11 * g0 - a01 * g1) / det;")],
    "no_renormalisation": [("double psi[3] = {r[0] / n, r[1] / n, r[2] / n};", "double psi[3] = {r[0], r[1], r[2]};")],
    "lambda_grows_on_accept": [("lambda /= 10.0;", "lambda *= 10.0;")],
    "accept_uphill": [("if (nxt.c < cur.c) {", "if (nxt.c > cur.c) {")],
    "bound_not_held": [("int hold_x = (px <= 0.0 && dx < 0.0) || (px >= W - 1.0 && dx > 0.0);", "int hold_x = 0;"),
                       ("int hold_y = (py <= 0.0 && dy < 0.0) || (py >= H - 1.0 && dy > 0.0);", "int hold_y = 0;")],
    "held_step_wrong_diagonal": [("else if (hold_x) { dx = 0.0; dy = -g1 / a11; }", "else if (hold_x) { dx = 0.0; dy = -g1 / a00; }"),
                                 ("else if (hold_y) { dy = 0.0; dx = -g0 / a00; }", "else if (hold_y) { dy = 0.0; dx = -g0 / a11; }")],
    "theta_is_chord": [("double th = 2.0 * asin(fmin(1.0, sqrt(cur.c) / 2.0));", "double th = sqrt(cur.c);")],
    "window_short": [("for (int dy = -C->r; dy <= C->r; ++dy) {", "for (int dy = -C->r; dy < C->r; ++dy) {")],
    "window_wrong_stride": [("int mx = mx0 + sp * dx;", "int mx = mx0 + dx;")],
    "tie_takes_last": [("if (s > best) { second = best; best = s; lev_m = m; }",
                        "if (s >= best) { second = best; best = s; lev_m = m; }")],
    "levels_same_spacing": [("const int sp = 1 << lev;", "const int sp = 1;")],
    "levels_centre_not_moved": [("        mx0 = (int)(lev_m % W);\n        my0 = (int)(lev_m / W);\n", "")],
    "refine_rounds_down": [("int mx0 = (int)floor(px + 0.5), my0 = (int)floor(py + 0.5);",
                            "int mx0 = (int)floor(px), my0 = (int)floor(py);")],
    "conf_gate_strict": [("sqrt(C->Qii[best_m] * C->Qji[n]) >= C->conf_min", "sqrt(C->Qii[best_m] * C->Qji[n]) > C->conf_min")],
    "conf_gate_wrong_pixel": [("sqrt(C->Qii[best_m] * C->Qji[n])", "sqrt(C->Qii[n] * C->Qji[n])")],
    "xhat_from_rays": [("bilerp3(C->Xii, &cl, C->xhat + 3 * n);", "bilerp3(C->rm.R, &cl, C->xhat + 3 * n);")],
    "ray_image_not_normalised": [("R[3 * m + 0] = x[0] / n;", "R[3 * m + 0] = x[0];"),
                                 ("R[3 * m + 1] = x[1] / n;", "R[3 * m + 1] = x[1];"),
                                 ("R[3 * m + 2] = x[2] / n;", "R[3 * m + 2] = x[2];")],
    "target_not_normalised": [("/* Target ray psi(x) (Sec. 3.1). */\n    double t[3] = {x[0] / xn, x[1] / xn, x[2] / xn};",
                               "/* Target ray psi(x) (Sec. 3.1). */\n    double t[3] = {x[0], x[1], x[2]};")],
    "identity_init_transposed": [("px0 = (double)(n % W);\n        py0 = (double)(n / W);",
                                  "px0 = (double)(n / W);\n        py0 = (double)(n % W);")],
    "bilinear_weights_swapped": [("w10 = c->a * (1 - c->b);", "w10 = (1 - c->a) * c->b;"),
                                 ("double w01 = (1 - c->a) * c->b,", "double w01 = c->a * (1 - c->b),")],
    "bwd_drops_direct_xhat_term": [("dXii[3 * cm[c] + k] += w[c] * gx[k];", "dXii[3 * cm[c] + k] += 0.0 * gx[k];")],
    "bwd_query_sign": [("for (int k = 0; k < 3; ++k) dXji[3 * n + k] = out[k];",
                        "for (int k = 0; k < 3; ++k) dXji[3 * n + k] = -out[k];")],
    "bwd_one_row_derivative": [("drx[k] = (1 - b) * (R10[k] - R00[k]) + b * (R11[k] - R01[k]);",
                                "drx[k] = (R10[k] - R00[k]);")],
    "bwd_drops_ray_norm": [("dXii[3 * cm[c] + k] -= (w[c] / rn) * out[k];", "dXii[3 * cm[c] + k] -= w[c] * out[k];")],
    "bwd_ignores_hold": [("int held_x = p[2 * n] <= 0.0 || p[2 * n] >= W - 1.0;", "int held_x = 0;"),
                         ("int held_y = p[2 * n + 1] <= 0.0 || p[2 * n + 1] >= H - 1.0;", "int held_y = 0;")],
    "bwd_corner_weights_swapped": [("double w[4] = {(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b};",
                                    "double w[4] = {(1 - a) * (1 - b), (1 - a) * b, a * (1 - b), a * b};")],
    "bwd_xhat_derivative_transposed": [("gp0 += dxx * gx[k];\n                gp1 += dxy * gx[k];",
                                        "gp0 += dxy * gx[k];\n                gp1 += dxx * gx[k];")],
}

# Edits of oracle/m3s_track_oracle.c; a third element True replaces every
# occurrence (the same expression appears in the solver and in the residual
# function).
TRACK_MUTANTS = {
    "track_rotation_jacobian_sign": [("J[i][3 + j] = -S[i][j] / d;", "J[i][3 + j] = S[i][j] / d;"),
                                     ("J[7 * i + 3 + j] = -S[i][j] / d;", "J[7 * i + 3 + j] = S[i][j] / d;")],
    "track_norm_jacobian_missing_1_over_d": [("J[i][j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]) / d;",
                                              "J[i][j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]);"),
                                             ("J[7 * i + j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]) / d;",
                                              "J[7 * i + j] = ((i == j ? 1.0 : 0.0) - u[i] * u[j]);")],
    "track_dist_scale_jacobian": [("J[3][6] = d;", "J[3][6] = 1.0;"), ("J[27] = d;", "J[27] = 1.0;")],
    "track_right_plus_update": [("        compose(E, T);\n",
                                 "        { double tmp[12]; memcpy(tmp, T, sizeof tmp); memcpy(T, E, sizeof tmp); compose(tmp, T); }\n")],
    "track_exp_without_V": [("tv += V * v[j];", "tv += (i == j ? 1.0 : 0.0) * v[j];")],
    "track_huber_weight_inverted": [("return a <= width ? 1.0 : width / a;", "return a <= width ? 1.0 : a / width;")],
    "track_confidence_gate_ignored": [("if (!(q > q_min)) continue;", "")],
    "track_weight_ignores_q": [("double w_ray = q / (sigma_ray * sigma_ray)", "double w_ray = 1.0 / (sigma_ray * sigma_ray)"),
                               ("double w_dist = q / (sigma_dist * sigma_dist)", "double w_dist = 1.0 / (sigma_dist * sigma_dist)")],
    "track_ray_residual_sign": [("double r[3] = {u[0] - Y[0] / dy, u[1] - Y[1] / dy, u[2] - Y[2] / dy};",
                                 "double r[3] = {Y[0] / dy - u[0], Y[1] / dy - u[1], Y[2] / dy - u[2]};")],
    "fuse_weights_swapped": [("(c_old * Xc[3 * n + k] + c_new * x[k])", "(c_new * Xc[3 * n + k] + c_old * x[k])")],
    "fuse_untransformed": [("+ c_new * x[k]) / c_sum", "+ c_new * X[3 * n + k]) / c_sum")],
    "fuse_confidence_not_summed": [("        Cc[n] = c_sum;\n", "        Cc[n] = c_new;\n")],
    "fuse_no_normalisation": [(") / c_sum;", ") / (c_sum + 1.0);")],
}

BACKEND_MUTANTS = {
    "backend_sign_of_i_jacobian": [("Ji[7 * a + b] = -s;", "Ji[7 * a + b] = s;")],
    "backend_adjoint_of_pose_not_inverse": [("bk_adjoint(Tii, A);", "bk_adjoint(Ti, A);")],
    "backend_relative_pose_order": [("bk_mul(Tii, Tj, Tij);", "bk_mul(Tj, Tii, Tij);")],
    "backend_adjoint_missing_cross_term": [("A[7 * i + 3 + j] = tr;", "A[7 * i + 3 + j] = 0.0;")],
    "backend_adjoint_scale_column_sign": [("A[7 * i + 6] = -t[i];", "A[7 * i + 6] = t[i];")],
    "backend_gauge_fixes_wrong_block": [("b[r] = -sys.g[7 + r];", "b[r] = -sys.g[r];")],
    "backend_no_cross_blocks": [("for (int c = 0; c < 2; ++c)", "for (int c = p; c <= p; ++c)")],
    "backend_right_update": [("bk_mul(E7, T_WC + 12 * k, Tn);", "bk_mul(T_WC + 12 * k, E7, Tn);")],
    "backend_inverse_scale": [("out[4 * i + j] = T[4 * j + i] / s2;", "out[4 * i + j] = T[4 * j + i] / s;")],
    "backend_measured_point_swapped": [("Xc + 3 * ((long)i * HW + m), r, Ji, Jj))", "Xc + 3 * ((long)i * HW + n), r, Ji, Jj))")],
}

_BATTERY = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import oracle, pins
lib = oracle.load(%(lib)r)
for pin in pins.ALL_PINS:
    try:
        pin(lib)
    except AssertionError as e:
        print("CAUGHT by", pin.__name__, "-", str(e)[:120]); sys.exit(0)
print("SURVIVED"); sys.exit(3)
"""


def _build_and_run(name, edits, tmpdir, which="match"):
    path = {"match": oracle._SRC, "track": oracle._TRACK_SRC, "backend": oracle._BACKEND_SRC}[which]
    src = open(path).read()
    for old, new in edits:
        assert src.count(old) == 1, "mutant %s: snippet not found exactly once: %r" % (name, old)
        src = src.replace(old, new)
    cpath = os.path.join(tmpdir, name + ".c")
    with open(cpath, "w") as f:
        f.write(src)
    out = os.path.join(tmpdir, "lib_" + name + ".so")
    if which == "match":
        lib = oracle.compile_oracle(cpath, out)
    elif which == "track":
        lib = oracle.compile_oracle(oracle._SRC, out, track_src=cpath)
    else:
        lib = oracle.compile_oracle(oracle._SRC, out, backend_src=cpath)
    code = _BATTERY % dict(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env)
    return name, r.returncode, (r.stdout + r.stderr).strip()[-400:]


def test_every_mutant_is_caught(tmp_path):
    jobs = ([(k, v, "match") for k, v in MUTANTS.items()] + [(k, v, "track") for k, v in TRACK_MUTANTS.items()] +
            [(k, v, "backend") for k, v in BACKEND_MUTANTS.items()])
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda j: _build_and_run(j[0], j[1], str(tmp_path), j[2]), jobs))
    survived = [(n, out) for n, rc, out in results if rc == 3]
    for n, rc, out in results:
        print("%-32s rc=%d %s" % (n, rc, out.splitlines()[-1] if out else ""))
    assert not survived, "mutants not caught by any pin: %s" % survived
