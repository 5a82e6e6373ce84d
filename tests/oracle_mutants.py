"""Mutation check of the oracle pins (run by hand, not collected by pytest).

Each entry plants one plausible mistake in a scratch copy of the oracle's C
source (a dropped or wrong term, a wrong sign, index or constant) and runs
the CPU pins against it; every mutant must make at least one pin fail.

    python tests/oracle_mutants.py            # all mutants
    python tests/oracle_mutants.py sf_x4      # one
"""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_bounds.py", "tests/test_oracle_pose5.py",
        "tests/test_oracle_refine.py"]

# (name, text in gv_oracle.c, replacement)
MUTANTS = [
    ("kappa_always_true", "if (rmin2 < C->Rg2) return 1; /* apex guard", "return 1; /* apex guard"),
    ("leaf_point_L2", "ldexp(1.0, -(C->L[j] + 1));\n    pt[j]", "ldexp(1.0, -(C->L[j] + 2));\n    pt[j]"),
    ("yaw_minus", "(M_PI / 2.0) + atan(pt[3])", "(M_PI / 2.0) - atan(pt[3])"),
    ("sf_x4", "C->sf[q] = p2floor(ep / (double)(C->ell + 1));",
     "C->sf[q] = 4.0 * p2floor(ep / (double)(C->ell + 1));"),
    ("pad_m3", "(double)((m + 1) * (C->ell + 1))", "(double)((m + 3) * (C->ell + 1))"),
    ("extra_level", "while (ldexp(C->E[j], -L) > ej) {", "while (ldexp(C->E[j], -L) >= 0.5 * ej) {"),
    ("sXi_x64", "C->sXi = p2floor(ek / (l1 * Bk * C->Fb));", "C->sXi = 64.0 * p2floor(ek / (l1 * Bk * C->Fb));"),
    ("padz_3eps", "C->padz = ceil((C->epsn[2] + ez * 0.5)", "C->padz = ceil((3.0 * C->epsn[2] + ez * 0.5)"),
    ("zhi_rmax", "int zhi_ok = (Thi >= 0.0) && ((al * al) * rmin2 <= Thi * Thi);",
     "int zhi_ok = (Thi >= 0.0) && ((al * al) * rmax2 <= Thi * Thi);"),
    ("zlo_rmin", "int zlo_ok = (Tlo <= 0.0) || ((ah * ah) * rmax2 >= Tlo * Tlo);",
     "int zlo_ok = (Tlo <= 0.0) || ((ah * ah) * rmin2 >= Tlo * Tlo);"),
    ("arc_swap", "if (cross2(elx, ely, bx, by) >= 0.0 && cross2(bx, by, ehx, ehy) >= 0.0) return 1;",
     "if (cross2(elx, ely, bx, by) >= 0.0 && cross2(ehx, ehy, bx, by) >= 0.0) return 1;"),
    ("sector3", "default: x0 = -Bhi; x1 = -Blo; y0 = Alo; y1 = Ahi; break;",
     "default: x0 = -Bhi; x1 = -Blo; y0 = -Ahi; y1 = -Alo; break;"),
    ("canon_step4", "for (int k = 0; k < nP; k++) fn = fn - tn[k] * u[P[k]];",
     "for (int k = 0; k < nP; k++) fn = fn + tn[k] * u[P[k]];"),
    ("canon_floor", "double fl = nearbyint(floc / sf) * sf;", "double fl = floor(floc / sf) * sf;"),
    ("digit_lsb", "int b = (digit >> (a - 1 - k)) & 1;", "int b = (digit >> k) & 1;"),
    ("tie_high", "return (count << C->B) | (mask - idx);", "return (count << C->B) | idx;"),
    ("group_noweight", "S[k].w += S[i].w;", "S[k].w += 0;"),
    ("pad_next", "if (gmax < clo - C->pad[m][q]) return 0;",
     "if (gmax < clo - C->pad[m + 1 < C->Lstar ? m + 1 : m][q]) return 0;"),
    ("plane_sign", "r->p[1] = -((y * C->E[1]) * C->inv[2]);", "r->p[1] = ((y * C->E[1]) * C->inv[2]);"),
    ("line_front", "r->p[4] = ((y - x * C->lo[0]) - C->lo[1]) * C->inv[1];",
     "r->p[4] = ((y + x * C->lo[0]) - C->lo[1]) * C->inv[1];"),
    ("ray_minaxis", "if (fabs(u[k]) > fabs(u[pi])) pi = k;", "if (fabs(u[k]) < fabs(u[pi])) pi = k;"),
    ("ray_front", "r->p[4 + qi] = ((w[q] - C->lo[q]) + s * (C->lo[pi] - w[pi])) * C->inv[q];",
     "r->p[4 + qi] = ((w[q] - C->lo[q]) + s * (C->lo[pi] + w[pi])) * C->inv[q];"),
    ("pose_eta", "r->p[4] = p->col[4][i] * C->ce;", "r->p[4] = p->col[4][i];"),
    ("sEta_x64", "C->sEta = p2floor(ez / (l1 * Rb * C->Fb));", "C->sEta = 64.0 * p2floor(ez / (l1 * Rb * C->Fb));"),
    ("sW_x64", "C->sW = p2floor(wz < wk ? wz : wk);", "C->sW = 64.0 * p2floor(wz < wk ? wz : wk);"),
    ("Rg_x4", "double Rg = ldexp(1.0, -Lxy); /* apex guard", "double Rg = ldexp(4.0, -Lxy); /* apex guard"),
    ("guard_rmax", "if (rmin2 < C->Rg2) return 1;", "if (rmax2 < C->Rg2) return 1;"),
    ("padk_3eps", "C->padk = ceil((C->epsk + ek * 0.5)", "C->padk = ceil((3.0 * C->epsk + ek * 0.5)"),
    ("inl_last", "if (inl && k < cap) inl[k] = i;", "if (inl && k < cap) inl[k] = i + (i == C->prob->n - 1);"),
    ("sim_front_d", "r->p[3] = (px * C->E[1]) * C->inv[3];", "r->p[3] = -(px * C->E[1]) * C->inv[3];"),
    # 5-DoF (unknown focal length)
    ("f5_zhi_Fh", "double ah = a * Fh, al = a * Fl;", "double ah = a * Fh, al = a * Fh;"),
    ("f5_zlo_Fl", "double ah = a * Fh, al = a * Fl;", "double ah = a * Fl, al = a * Fl;"),
    ("f5_t_swap", "double tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;",
     "double tl = t1 < t2 ? t2 : t1, th = t1 < t2 ? t1 : t2;"),
    ("f5_cell_hi", "Fh = C->flo + C->Ef * ((double)(cc[4] + 1) * hf);",
     "Fh = C->flo + C->Ef * ((double)(cc[4] + 2) * hf);"),
    ("f5_cell_lo", "Fl = C->flo + C->Ef * ((double)cc[4] * hf);", "Fl = C->flo + C->Ef * ((double)(cc[4] + 1) * hf);"),
    ("f5_no_f", "if (C->fam == OR_POSE5DOF) {\n    double hf", "if (0) {\n    double hf"),
    ("f5_sEta_noF", "C->sEta = p2floor(ez / (l1 * Rb * C->Fb));", "C->sEta = p2floor(ez / (l1 * Rb));"),
    ("f5_sXi_noF", "C->sXi = p2floor(ek / (l1 * Bk * C->Fb));", "C->sXi = p2floor(ek / (l1 * Bk));"),
    ("f5_wz_noF", "double wz = ez / (l1 * Hb * C->Fb)", "double wz = ez / (l1 * Hb)"),
    # verification and refinement after the vote
    ("rf_kappa_sign", "dd[3][0] = d[1] / n2; dd[3][1] = -d[0] / n2;", "dd[3][0] = -d[1] / n2; dd[3][1] = d[0] / n2;"),
    ("rf_no_fder", "for (int c = 0; c < 3; c++) J[c][4] = -((dof[c] - oh[c] * pr) / no);",
     "for (int c = 0; c < 3; c++) J[c][4] = 0.0 * pr;"),
    ("rf_tau0", "round == 0 ? T20 : T2", "T2"),
    ("rf_rot1", "case 1: *u1 = b; *u2 = -a; break;\n    case 2: *u1 = -a", "case 1: *u1 = -b; *u2 = a; break;\n    case 2: *u1 = -a"),
    ("rf_obs_s", "o[2] = b * sqrt(1.0 + a * a);", "o[2] = b;"),
    ("rf_dx_sign", "rf_rot(s, -1.0, 0.0, &ux1, &ux2);", "rf_rot(s, 1.0, 0.0, &ux1, &ux2);"),
    ("sim_axes", "*nP = 2; P[0] = 0; P[1] = 1; *nQ = 2; Q[0] = 2; Q[1] = 3;",
     "*nP = 2; P[0] = 0; P[1] = 1; *nQ = 2; Q[0] = 3; Q[1] = 2;"),
]


def run(name, old, new):
    with tempfile.TemporaryDirectory(prefix=f"mut_{name}_") as d:
        for sub in ("oracle", "tests", "paper_2107_11810_amd"):
            shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                            ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), d)
        src_path = os.path.join(d, "oracle", "gv_oracle.c")
        src = open(src_path).read()
        if src.count(old) != 1:
            return None, f"pattern found {src.count(old)} times"
        open(src_path, "w").write(src.replace(old, new))
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                           + PINS, cwd=d, capture_output=True, text=True)
        tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-200:]
        return r.returncode != 0, tail


def main():
    only = set(sys.argv[1:])
    survived = []
    for name, old, new in MUTANTS:
        if only and name not in only:
            continue
        killed, tail = run(name, old, new)
        print(f"{name:20s} {'killed' if killed else 'SURVIVED' if killed is False else 'NOT APPLIED'}  {tail}",
              flush=True)
        if not killed:
            survived.append(name)
    sys.exit(1 if survived else 0)


if __name__ == "__main__":
    main()
