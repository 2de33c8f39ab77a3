"""The oracle's pins must catch plausible mistakes: each mutant below plants
one (a dropped term, a sign, a transposed operand, a wrong constant) in a
scratch copy of the oracle source, builds it with gcc on the CPU, and runs
the oracle pin tests against it; every mutant must make them fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_kernel_projection.py", "tests/test_oracle_render.py",
             "tests/test_oracle_grad_bin.py", "tests/test_oracle_gaussian_sh.py"]

MUTANTS = {
    "mean2d_adjoint_sign": ("sa.mean2d[0] = -adj_r2 * 2.0", "sa.mean2d[0] = adj_r2 * 2.0"),
    "quat_w_adjoint": ("dq[0] = 2.0 * (-z * dR[1]", "dq[0] = 2.0 * (z * dR[1]"),
    "jacobian_tz_adjoint": ("+ dJ[4] * (-fy / (tz * tz))", "+ dJ[4] * (fy / (tz * tz))"),
    "dropped_transmittance_term": ("adjT = adjT * (1.0 - e->alpha) + gc * e->alpha;",
                                   "adjT = adjT * (1.0 - e->alpha);"),
    "lobe_theta_phi_swap": ("adj_x * (dR_dth[0] * f->vdir[0]", "adj_x * (dR_dph[0] * f->vdir[0]"),
    "camera_centre_transposed": ("campos[k] = -(W[k] * cam->t[0] + W[3 + k]",
                                 "campos[k] = -(W[3*k] * cam->t[0] + W[3 * k+1]"),
    "pixel_centre": ("pix_xy[2 * p] + 0.5, pix_xy[2 * p + 1] + 0.5,\n                                    alpha_max",
                     "pix_xy[2 * p] + 0.0, pix_xy[2 * p + 1] + 0.5,\n                                    alpha_max"),
    "jacobian_sign": ("f->Jm[2] = -cam->fx * tx / (tz * tz);", "f->Jm[2] = cam->fx * tx / (tz * tz);"),
    "view_rotation_transposed": ("acc += f->Jm[3 * a + k] * W[3 * k + b];",
                                 "acc += f->Jm[3 * a + k] * W[3 * b + k];"),
    "kernel_constant": ("f->beta = s->sh ? 0.0 : 4.0 * exp(s->betas[i]);",
                        "f->beta = s->sh ? 0.0 : 3.5 * exp(s->betas[i]);"),
    "gaussian_exponent": ("B = exp(-0.5 * r2);", "B = exp(-r2);"),
    "gaussian_cutoff": ("if (!(r2 < 9.0)) continue;", "if (!(r2 < 4.0)) continue;"),
    "gaussian_extent": ("double ext = s->sh ? 3.0 : 1.0;", "double ext = s->sh ? 2.0 : 1.0;"),
    "sh_legendre_phase": ("case 21: return -3.0 * x * s;", "case 21: return 3.0 * x * s;"),
    "sh_offset": ("double acc = 0.5;", "double acc = 0.0;"),
    "view_direction_sign": ("double v[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};",
                            "double v[3] = {campos[0] - mu[0], campos[1] - mu[1], campos[2] - mu[2]};"),
    "quaternion_sign": ("R[1] = 2.0 * (x * y - w * z);", "R[1] = 2.0 * (x * y + w * z);"),
    "termination_rule": ("        last = i;\n        if (T < t_eps) break;",
                         "        last = i;\n        if (T_prev * (1.0 - a) < t_eps * 0.5) break;"),
    "scale_adjoint_factor": ("add_grad(g->scales, 3 * i + c, 2.0 * sc[c] * acc);",
                             "add_grad(g->scales, 3 * i + c, sc[c] * acc);"),
    "non_finite_not_culled": ("    if (!params_finite(s, i)) return;\n", ""),
    "lobe_beta_not_checked": ("        if (!isfinite(s->lobe_betas[l])) return 0;\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, oracle):
    src = open(os.path.join(ROOT, "oracle", "dbs_oracle.c")).read()
    before, after = MUTANTS[name]
    assert src.count(before) >= 1, "mutation site not found"
    (tmp_path / "m.c").write_text(src.replace(before, after, 1))
    lib = str(tmp_path / "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", lib,
                           str(tmp_path / "m.c"), "-lm"])
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + PIN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, r.stdout[-2000:]
