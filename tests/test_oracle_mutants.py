"""The pins are strong enough: each plausible mistake planted in a copy of the oracle (on the
CPU, in a temporary build) makes at least one pin of the oracle fail."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# (what the mistake is, text in the oracle, replacement)
MUTANTS = [
    ("bed correction dropped", "*pl = 0.5 * g * (hl * hl - hsl * hsl);", "*pl = 0.0;"),
    ("reconstruction uses the other bed", "double hsl = fmax(0.0, hl - (zs - zl));",
     "double hsl = fmax(0.0, hl - (zs - zr));"),
    ("momentum rotated back with a wrong sign", "f[1] = fq * nx - fw * ny;\n    f[2] = fq * ny + fw * nx;\n}\n\nstatic",
     "f[1] = fq * nx + fw * ny;\n    f[2] = fq * ny + fw * nx;\n}\n\nstatic"),
    ("dry-right front speed u + c", "*sr = ql + 2.0 * cl;", "*sr = ql + cl;"),
    ("star velocity sound-speed term swapped", "(ql + qr) / 2.0 + (cl - cr)", "(ql + qr) / 2.0 + (cr - cl)"),
    ("star sound speed velocity term swapped", "(cl + cr) / 2.0 + (ql - qr) / 4.0", "(cl + cr) / 2.0 + (qr - ql) / 4.0"),
    ("HLL jump term sign", "+ sl * sr * (hr - hl)) / den", "- sl * sr * (hr - hl)) / den"),
    ("HLL momentum jump uses velocities", "sl * sr * (hr * qr - hl * ql)", "sl * sr * (qr - ql)"),
    ("contact upwinding inverted", "const double wup = sstar > 0.0 ? wl : (sstar < 0.0 ? wr",
     "const double wup = sstar > 0.0 ? wr : (sstar < 0.0 ? wl"),
    ("hydrostatic pressure without the half", "fql = hl * ql * ql + 0.5 * g * hl * hl", "fql = hl * ql * ql + g * hl * hl"),
    ("wall ghost keeps the normal velocity", "om_hllc_normal(g, hs, q, w, hs, -q, w,", "om_hllc_normal(g, hs, q, w, hs, q, w,"),
    ("friction depth exponent 1/3 short", "(hs * hs * cbrt(hs))", "(hs * cbrt(hs))"),
    ("friction linear in n", "dt * g * n[c] * n[c] * mag", "dt * g * n[c] * mag"),
    ("Euler update sign", "double hs = h[c] - r * acc[0];", "double hs = h[c] + r * acc[0];"),
    ("x-momentum update sign", "const double hus = hu[c] - r * acc[1];", "const double hus = hu[c] + r * acc[1];"),
    ("last edge of y-momentum dropped", "acc[2] = acc[2] + c2;", "acc[2] = acc[2];"),
    ("neighbour side not negated", "const double s = (m->edge_l[e] == c) ? 1.0 : -1.0;\n            const double pk = (m->edge_l[e] == c) ? w->pl[e] : w->pr[e];",
     "const double s = 1.0;\n            const double pk = (m->edge_l[e] == c) ? w->pl[e] : w->pr[e];"),
    ("inradius A/P", "m->inradius[c] = 2.0 * a / (l0 + l1 + l2);", "m->inradius[c] = a / (l0 + l1 + l2);"),
    ("CFL ignores the flow speed", "s = sqrt(u * u + v * v) + sqrt(p->g * h[c]);", "s = sqrt(p->g * h[c]);"),
    ("CFL misses the Courant number", "return p->courant * best;", "return best;"),
    ("normal points inward", "*nx = dy / l;\n    *ny = -dx / l;", "*nx = -dy / l;\n    *ny = dx / l;"),
    ("dry cells keep momentum", "hu[c] = 0.0;\n            hv[c] = 0.0;", "hu[c] = hus;\n            hv[c] = hvs;"),
    ("inflow sign", "f[0] = -q_in;", "f[0] = q_in;"),
    ("inflow momentum without the half", "const double mom = q_in * q_in / hb + 0.5 * g * hb * hb;",
     "const double mom = q_in * q_in / hb + g * hb * hb;"),
    ("inflow boundary depth is the cell depth", "const double hb = fmax(h, hc);", "const double hb = h;"),
    ("inflow speed without the flow term", "return q_in / hb + sqrt(g * hb);", "return sqrt(g * hb);"),
    ("CFL ignores the inflow speed", "if (sb > s) s = sb;", "(void)sb;"),
    ("t_end clip ignored", "if (t_end > 0.0 && dt >= t_end - st->t) { dt = t_end - st->t; last = 1; }",
     "if (t_end > 0.0 && dt >= t_end - st->t) { last = 1; }"),
]

PINS = [os.path.join(HERE, "test_oracle_flux.py"), os.path.join(HERE, "test_oracle_physics.py")]


def _check(mut, tmp):
    name, old, new = mut
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
    path = os.path.join(tmp, f"m{abs(hash(name))}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = path[:-2] + ".so"
    oracle.build(path, so)
    env = dict(os.environ, SWE_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(4) as ex:
            results = list(ex.map(lambda m: _check(m, tmp), MUTANTS))
    survivors = [n for n, rc in results if rc == 0]
    assert not survivors, f"mistakes no pin catches: {survivors}"
