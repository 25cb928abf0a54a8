"""Shared comparison of a device run with the oracle (imported by the GPU
parity tests; not collected itself).

Every field f is compared over the interior cells in two norms, each
normalised by the field's own scale s_f = max(max |f_oracle|, floor_f):

  relative L1   sum |f_gpu - f_oracle| / max(sum |f_oracle|, N s_f)
  element-wise  max |f_gpu - f_oracle| / s_f

The floors only matter for fields that vanish or nearly vanish.  u~: 1e-3;
the implicit solve stops once its Newton step is below newton_tol (1 +
max|u~|) W^2 (1e-13 for slow flows), so a velocity far below 1 is fixed only
to ~1e-13 absolute on either side, and with this floor the element-wise bound
1e-9 admits 1e-12 absolute (a cold, heavy fluid pushed by the field, as in
the telegraph test, moves at |u~| ~ 1e-7).  p: 1e-6 max rho (the recovery
forms p from a difference of terms of size rho, so its round-off is ~1e-16
rho).  E and the face fields: 1e-12 of the largest component.  The true
relative L1 (sum |diff| / sum |f_oracle|) is printed beside them.
"""
import sys

import numpy as np

NAMES = ["rho", "u~x", "u~y", "u~z", "p", "Ex", "Ey", "Ez", "Bx", "By", "Bz"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_E(run):
    """contravariant E of a device run, q_E / psi^6 (host side)"""
    q = run.cons()
    ps6 = 1.0 if not run.setup.metric else run.setup.psi ** 6
    return q[5:8] / ps6


def oracle_E(ref):
    ps6 = 1.0 if ref.psi is None else ref.psi ** 6
    return np.stack([ref.q[5 + v] / ps6 for v in range(3)])


def _err(a, b, floor):
    s = max(float(np.abs(b).max()) if b.size else 0.0, floor)
    d = np.abs(a - b)
    den = max(float(np.abs(b).sum()), b.size * s)
    true = float(d.sum() / np.abs(b).sum()) if np.abs(b).sum() > 0 else 0.0
    return float(d.sum() / den), float(d.max() / s) if s > 0 else 0.0, true


def state_errors(s, got_prim, ref_prim, got_E, ref_E, got_face, ref_face):
    """[(name, rel_l1, max_rel, true_rel_l1)] over primitives, E and faces"""
    sl = s.interior
    out = []
    rho_max = float(np.abs(ref_prim[0][sl]).max())
    for v in range(5):
        floor = 0.0 if v == 0 else (1e-3 if v < 4 else 1e-6 * rho_max)
        out.append((NAMES[v],) + _err(got_prim[v][sl], ref_prim[v][sl], floor))
    bsc = max(float(np.abs(ref_face[d][sl]).max()) for d in range(3))
    esc = max(float(np.abs(ref_E[i][sl]).max()) for i in range(3))
    em = max(bsc, esc, 1e-300)
    for i in range(3):
        out.append((NAMES[5 + i],) + _err(got_E[i][sl], ref_E[i][sl], 1e-12 * em))
    for d in range(3):
        out.append((NAMES[8 + d],) + _err(got_face[d][sl], ref_face[d][sl], 1e-12 * max(bsc, 1e-300)))
    return out


def check(s, run, ref, tol_l1, tol_max, tag=""):
    """compare a device Run with an OracleState; print and assert both norms"""
    errs = state_errors(s, run.prims(), ref.prim, device_E(run), oracle_E(ref), run.faces(), ref.face)
    say("  %s rel L1 max %.1e, element-wise max %.1e (%s; true rel L1 %s)" % (
        tag, max(e[1] for e in errs), max(e[2] for e in errs),
        ", ".join("%s %.0e/%.0e" % (n, a, m) for n, a, m, _ in errs),
        " ".join("%.0e" % e[3] for e in errs)))
    bad = [e for e in errs if not (e[1] <= tol_l1 and e[2] <= tol_max)]
    assert not bad, bad
    return errs
