"""Planted mistakes in the oracle (CPU only): every one must fail a pin.

Each case copies oracle/pcpic_oracle.c, makes one plausible mistake in it (a
dropped or doubled term, a wrong sign, index or factor, a transposed operand),
builds the copy and runs the pins against it in a child process.  The pins
that face the paper and the mathematics (test_oracle_pins.py) must catch every
mistake in the forward step; the finite-difference pins of the gradient
(test_oracle_adjoint.py) must catch every mistake in the reverse sweep; the GR
pins (test_oracle_gr.py) every mistake in the lapse factors of the GR step.  The
unmodified oracle passes both files in the main run.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pcpic_oracle.c")

pytestmark = pytest.mark.slow

# (what is planted, original text, mutated text)
FORWARD = [
    ("sign of the E_z term in the B_phi update (eq. 3)",
     "k->dtR * st->ez[i]);", "-k->dtR * st->ez[i]);"),
    ("mirror factor 2 dropped in the E_r update at node N",
     "st->er[N] = st->er[N] + k->tw * st->b[N - 1];", "st->er[N] = st->er[N] + k->dtdz * st->b[N - 1];"),
    ("mirror-doubled node-N weight dropped in the Poisson right-hand side",
     "int64_t wi = (i == N) ? 2 * st->w[i] : st->w[i];", "int64_t wi = st->w[i];"),
    ("mirror row of the Poisson matrix not doubled",
     "double a = (i == N) ? 2.0 : 1.0;", "double a = 1.0;"),
    ("gather between nodes instead of faces",
     "double s = x - 0.5, E;", "double s = x, E;"),
    ("move with u instead of v = u / gamma",
     "            v = u1 / gam;\n            x1 = x + k->dtdz * v;", "            v = u1 / gam;\n            x1 = x + k->dtdz * u1;"),
    ("cumulative weight off by one cell",
     "if (cell > i) return 0;", "if (cell > i + 1) return 0;"),
    ("sign of the background term of the surface field",
     "double es = st->ez[0] - k->fourpi * (t1 - t2);", "double es = st->ez[0] - k->fourpi * (t1 + t2);"),
    ("whole cell instead of half cell in the node-0 Gauss law",
     "k->hdz = 0.5 * k->dz;", "k->hdz = k->dz;"),
    ("frame dragging with eta^2 instead of eta^3 (eq. 7)",
     "double fd = 1.0 - c->kappa / e3;", "double fd = 1.0 - c->kappa / (eta * eta);"),
    ("sign of the current term of the E_z update",
     "st->ez[i] = (st->ez[i] + k->dtR * st->b[i]) - k->c4 * (double)st->j[i];",
     "st->ez[i] = (st->ez[i] + k->dtR * st->b[i]) + k->c4 * (double)st->j[i];"),
    ("node-0 weight of a particle in cell 0 taken from the wrong side",
     "            t->w0 += k->oneP - F1;", "            t->w0 += F1;"),
    ("inclination term of eq. 6 growing as eta instead of eta^(1/2)",
     "double br = fd + s * sqrt(eta);", "double br = fd + s * eta;"),
    ("redshift with r_g r instead of r_g / r",
     "double al = sqrt(1.0 - c->rg_over_rstar / eta);", "double al = sqrt(1.0 - c->rg_over_rstar * eta);"),
    ("steady start drifting with u instead of v",
     "double x1 = k.gr ? x + k.dtdz * (orc_alpha2(c, x * k.dz) * v) : x + k.dtdz * v;",
     "double x1 = k.gr ? x + k.dtdz * (orc_alpha2(c, x * k.dz) * v) : x + k.dtdz * u;"),
    ("steady start B = J / (R dt) without the 4 pi q_m 2^-P factor",
     "st->b[i] = (k.c4 * (double)st->j[i]) / k.dtR;", "st->b[i] = ((double)st->j[i]) / k.dtR;"),
    ("sin(i) instead of tan(i) after dividing eq. 6 by cos(i)",
     "((1.5 * c->theta_star) * tan(c->incl))", "((1.5 * c->theta_star) * sin(c->incl))"),
]

# the lapse alpha of the full-GR step (GR_ALPHA), against the GR pins
GR = [
    ("sign of the gravity term in the GR kick",
     "u1 = u + (al * E - kg * gh);", "u1 = u + (al * E + kg * gh);"),
    ("GR move with v instead of alpha^2 v",
     "x1 = x + k->dtdz * (a2h * v);", "x1 = x + k->dtdz * v;"),
    ("gravity with gamma(u) instead of the midpoint gamma",
     "u1 = u + (al * E - kg * gh);", "u1 = u + (al * E - kg * g0);"),
    ("surface field without rho_GJ,0 / alpha_0",
     "if (k->gr) t2 = t2 / orc_alpha_node(c, k->dz, 0);", "if (k->gr) t2 = t2;"),
    ("alpha_{i+1/2} dropped from the B term of the E_z update",
     "st->ez[i] = (st->ez[i] + k->dtR * (orc_alpha_face(c, dz, i) * st->b[i])) - k->c4 * jw;",
     "st->ez[i] = (st->ez[i] + k->dtR * st->b[i]) - k->c4 * jw;"),
    ("alpha_i dropped from the E_r update",
     "st->er[i] = st->er[i] - k->dtdz * (orc_alpha_node(c, dz, i) * d);", "st->er[i] = st->er[i] - k->dtdz * d;"),
    ("alpha dropped on E_r in the B update",
     "double d = orc_alpha_node(c, dz, i + 1) * st->er[i + 1] - orc_alpha_node(c, dz, i) * st->er[i];",
     "double d = st->er[i + 1] - st->er[i];"),
    ("Poisson right-hand side with rho_GJ instead of rho_GJ / alpha",
     "double rg = k.gr ? st->rho_gj[i] / orc_alpha_node(c, k.dz, i) : st->rho_gj[i];", "double rg = st->rho_gj[i];"),
    ("E_r = Phi / R instead of Phi / (alpha R) at the start",
     "st->er[i] = (k.gr ? st->phi[i] / orc_alpha_node(c, k.dz, i) : st->phi[i]) / c->radius;",
     "st->er[i] = st->phi[i] / c->radius;"),
    ("alpha at faces taken at the node below (half a cell off)",
     "    return sqrt(orc_alpha2(c, ((double)i + 0.5) * dz));", "    return sqrt(orc_alpha2(c, (double)i * dz));"),
    ("alpha^2 on the wrong side in the Poisson diagonal",
     "double bd = k.gr ? -(2.0 + h2 / orc_alpha2(c, (double)i * k.dz)) : bdiag;",
     "double bd = k.gr ? -(2.0 + h2 * orc_alpha2(c, (double)i * k.dz)) : bdiag;"),
]

REVERSE = [
    ("d v / d u taken as 1/gamma instead of 1/gamma^3",
     "const double lu1t = lu1 + lx1 * k->dtdz / (gam * gam * gam);", "const double lu1t = lu1 + lx1 * k->dtdz / gam;"),
    ("sign of the deposit's position adjoint",
     "if (q->c1 >= 0 && q->c1 < N) lx1 += twoP * (wcls * lj[q->c1]);",
     "if (q->c1 >= 0 && q->c1 < N) lx1 -= twoP * (wcls * lj[q->c1]);"),
    ("kick-array adjoint dropped from the E_z adjoint",
     "const double a = lez[i] - k->dtR * lbp[i] + k->qmdt * lk[i];", "const double a = lez[i] - k->dtR * lbp[i];"),
    ("mirror factor dropped in the transposed E_r update",
     "double c = (i <= N - 1) ? ((i == N - 1) ? 2.0 : 1.0) : 0.0;", "double c = (i <= N - 1) ? 1.0 : 0.0;"),
    ("E_r neighbour term dropped in the B adjoint",
     "        if (i + 1 <= N - 1) a += k->dtdz * ler[i + 1];", "        if (i + 1 <= N - 1) a += 0.0 * ler[i + 1];"),
    ("gather-slope term dropped from the position adjoint",
     "*lx = lx1 + lx0J + lu1t * q->dEdx;", "*lx = lx1 + lx0J;"),
    ("loss seed d gamma / d u replaced by 1 / gamma",
     "lu1 = nex > 0 ? (q.u1 / q.gam) / (double)nex : 0.0;", "lu1 = nex > 0 ? (1.0 / q.gam) / (double)nex : 0.0;"),
]


def _run_case(tmp, idx, old, new, test_file):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {old}"
    d = os.path.join(tmp, f"m{idx}")
    os.makedirs(d, exist_ok=True)
    msrc = os.path.join(d, "pcpic_oracle.c")
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle import build_oracle
    lib = build_oracle.build(src=msrc, out=os.path.join(d, "liboracle.so"))
    env = dict(os.environ, PCPIC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", test_file)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-400:]


@pytest.mark.parametrize("cases,test_file", [(FORWARD, "test_oracle_pins.py"), (REVERSE, "test_oracle_adjoint.py"),
                                             (GR, "test_oracle_gr.py")],
                         ids=["forward-step", "reverse-sweep", "gr-alpha"])
def test_every_planted_mistake_fails_a_pin(tmp_path, cases, test_file):
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = [ex.submit(_run_case, str(tmp_path), k, old, new, test_file) for k, (_, old, new) in enumerate(cases)]
        results = [f.result() for f in futs]
    survivors = [(what, out) for (what, _, _), (rc, out) in zip(cases, results) if rc == 0]
    assert not survivors, "mistakes no pin catches: " + "; ".join(w for w, _ in survivors)
    # a failure must come from a failing pin, not from a crash of the child run
    for (what, _, _), (rc, out) in zip(cases, results):
        assert rc == 1, f"{what}: child pytest exited with {rc}: {out}"
