"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each case edits one plausible mistake (a dropped term, a wrong sign, a
wrong index, a transposed operand) into a temporary copy of
``oracle/phicomb_oracle.c``, builds it, and runs a compact battery of the
exact-reference pins through it.  At least one pin must fail.  The real
oracle source is never modified.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import refs
import workloads as wl

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "phicomb_oracle.c")

MUTATIONS = [
    ("no reordering of V",
     "static int perm_index(int b, int p) { return b == 0 ? 0 : p + 1 - b; }",
     "static int perm_index(int b, int p) { (void)p; return b; }"),
    ("shift sign in A_1",
     "y[i] = y[i] - xi * x[i];", "y[i] = y[i] + xi * x[i];"),
    ("undo factor sign",
     "mu[i] = exp(xi * t[i] / ssd);", "mu[i] = exp(-xi * t[i] / ssd);"),
    ("J step without /s (R1)",
     "            js[bb * P1 + bb + 1] = Dl[i] / ssd;\n    }\n    memcpy(S, Vb",
     "            js[bb * P1 + bb + 1] = Dl[i];\n    }\n    memcpy(S, Vb"),
    ("Jtilde dropped (identity)",
     "        small_expm_nilpotent(Nm, P1, jt);",
     "        for (int a = 0; a < P1 * P1; ++a) Nm[a] = 0.0;\n        small_expm_nilpotent(Nm, P1, jt);"),
    ("transposed dense operand",
     "                acc += row[j] * x[j];", "                acc += A->dense[j * n + i] * x[j];"),
    ("weight index without the permutation",
     "const double wgt = (form == 0) ? beta[i * P1 + perm_index(b, p)] : 1.0;",
     "const double wgt = (form == 0) ? beta[i * P1 + b] : 1.0;"),
    ("v_0 dropped from the recovery of exp(tA/s) v_0",
     "fc[q] = y[q] * t[i] + w0 * V[q];", "fc[q] = y[q] * t[i];"),
    ("last block not refreshed from S",
     "f2[q] = (p >= 1) ? e2[q] + sp[q] : e2[q];", "f2[q] = e2[q];"),
    ("recovery term without 1/k",
     "fc[z] = y[z] * ts / (double)kk;", "fc[z] = y[z] * ts;"),
    ("S-series term without t_i/s",
     "                const double ts = t[i] / ssd;\n                apply_A1(A, xi, dc, y);",
     "                const double ts = t[i];\n                apply_A1(A, xi, dc, y);"),
    ("alpha-form combine without Delta",
     "F[(int64_t)(r + i) * n + q] * Dl[i];", "F[(int64_t)(r + i) * n + q];"),
    ("s0 from one ratio too many",
     "s0 = exp(sum / (double)(r - jr));", "s0 = exp(sum / (double)(r - jr + 1));"),
    ("guard without the log cushion",
     "if (Lk + 0.5 * log(k + 1.0) + lmax > gmax || Lk < gmin)",
     "if (Lk + lmax > gmax || Lk < gmin)"),
    ("shift recovered with the wrong sign",
     "out->shift = -zs * s0;", "out->shift = zs * s0;"),
    ("objective power order reversed",
     "        coef[k] = c->b[k] * pw;", "        coef[m - k] = c->b[k] * pw;"),
]


def _diag_op(lams):
    n = len(lams)
    return wl.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                  np.asarray(lams, dtype=np.float64))


def _battery(orc):
    """Return the list of failed pin names (empty = all pass)."""
    failed = []

    def check(name, ok):
        if not ok:
            failed.append(name)

    # 1. small non-normal dense, general weights, several recovery steps
    try:
        pr = wl.small_problem(6, 3, 2, 1, t_scale=6.0, spread=4.0)
        ex = refs.exact_dense_mp(pr.op.A, pr.t, pr.beta, pr.V, dps=30)
        W, st, _ = orc.full(pr)
        check("dense-general", st["s_int"] >= 2 and refs.rel2_cols(W, ex).max() <= 1e-11)
        # 2. Vandermonde weights through the literal alpha-form
        pr = wl.small_problem(6, 3, 2, 2, t_scale=6.0, spread=4.0, vandermonde_weights=True)
        ex = refs.exact_dense_mp(pr.op.A, pr.t, pr.beta, pr.V, dps=30)
        prm = orc.params(pr.op, pr.tol, pr.v)
        Wa, _ = orc.solve(pr.op, pr.p, pr.r, pr.t, None, pr.V, pr.tol, prm["shift"], prm["s"],
                          form="alpha", alpha=pr.alpha)
        check("dense-alpha", refs.rel2_cols(Wa, ex).max() <= 1e-11)
    except Exception:
        failed.append("dense-exception")
    # 3. Laplacian with several recovery steps against the DST closed form
    try:
        pr = wl.config1()
        t = pr.t * 40
        prm = orc.params(pr.op, pr.tol, pr.v)
        W, st = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
        check("lap-dst", refs.rel2(W, refs.dst_laplacian(pr.op, t, pr.beta, pr.V)) <= 1e-13)
    except Exception:
        failed.append("lap-exception")
    # 4. scaled identity: s0 = c, guard index from the paper's inequality
    try:
        lc = 20.26
        op = _diag_op([math.exp(lc)] * 5)
        prm = orc.params(op, 2.0 ** -53, np.arange(1.0, 6.0))
        lmax = max(math.lgamma(62) - math.lgamma(j + 1) - math.lgamma(62 - j) for j in range(62))
        gmax = 0.8 * math.log(np.finfo(float).max)
        k_exp = max(k for k in range(1, 62) if lc * k + 0.5 * math.log(k + 1) + lmax <= gmax)
        check("cI-guard", prm["r_acc"] == k_exp)
        check("cI-s0", abs(prm["s0"] / math.exp(lc) - 1) < 1e-12)
        prm4 = orc.params(op, 2.0 ** -53, np.arange(1.0, 6.0), m=4)
        check("cI-shift", abs(prm4["shift"] / math.exp(lc) - 1) < 1e-3)
        # two-point spectrum {-c, 0}: f(z)^(2m) = ((z-1)^(2m) + z^(2m))/2, z* = 1/2
        c = 300.0
        op2 = _diag_op([-c] * 4 + [0.0] * 4)
        prm2 = orc.params(op2, 1e-10, np.ones(8), m=4)
        check("two-point-shift", abs(prm2["shift"] / (-0.5 * c) - 1) < 1e-3)
    except Exception:
        failed.append("cI-exception")
    return failed


@pytest.fixture(scope="module")
def original_source():
    with open(SRC) as f:
        return f.read()


def test_unmutated_battery_passes(orc):
    assert _battery(orc) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(orc, tmp_path, original_source, name, old, new):
    assert original_source.count(old) == 1, f"mutation anchor not unique/not found: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(original_source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=gnu11", "-fPIC", "-shared",
                           "-w", "-o", str(lib), str(src), "-lm"])
    with orc.using_library(str(lib)):
        failed = _battery(orc)
    assert failed, f"planted mistake '{name}' passed every pin"


# ------------------------------------------------------------- complex oracle
ZSRC = os.path.join(os.path.dirname(SRC), "phicomb_oracle_complex.c")

ZMUTATIONS = [
    ("S-series step with Re t", "const zc ts = t[i] / ssd;", "const zc ts = creal(t[i]) / ssd;"),
    ("undo factor with conj(xi)", "mu[i] = cexp(xi * t[i] / ssd);",
     "mu[i] = cexp(conj(xi) * t[i] / ssd);"),
    ("block norm of real parts", "s += cabs(X[(int64_t)q * n + i]);",
     "s += fabs(creal(X[(int64_t)q * n + i]));"),
    ("recovery of v_0 with conj(t)", "fc[q] = y[q] * t[i] + w0 * V[q];",
     "fc[q] = y[q] * conj(t[i]) + w0 * V[q];"),
    ("J step with conj(xi)", "js[bb * P1 + bb] = (-xi * t[i]) / ssd;",
     "js[bb * P1 + bb] = (-conj(xi) * t[i]) / ssd;"),
    ("Delta = conj(alpha)", "Dl[i] = (form == 1) ? alpha[i] : 1.0;",
     "Dl[i] = (form == 1) ? conj(alpha[i]) : 1.0;"),
    ("conjugated dense operand", "acc += row[j] * x[j];", "acc += conj(row[j]) * x[j];"),
    ("s_int from |Re t|", "if (cabs(t[i]) > tmax)\n            tmax = cabs(t[i]);",
     "if (fabs(creal(t[i])) > tmax)\n            tmax = fabs(creal(t[i]));"),
    ("conjugated weight table", "const zc wgt = (form == 0) ? beta[i * P1 + zperm(bl, p)] : 1.0;",
     "const zc wgt = (form == 0) ? conj(beta[i * P1 + zperm(bl, p)]) : 1.0;"),
]


def _zbattery(orc):
    """Compact complex pins; returns the names of the failed ones."""
    import test_oracle_complex as tz
    failed = []
    for name, fn, args in [
        ("z-diag", tz.test_complex_diagonal_closed_form, (1, 10.0)),
        ("z-dense", tz.test_complex_dense_against_augmented_exponential, (7, 5, 3, 1, 8.0)),
        ("z-real", tz.test_complex_path_on_real_data_equals_real_oracle, ()),
        ("z-imag", tz.test_complex_purely_imaginary_data, ()),
    ]:
        try:
            fn(orc, *args)
        except Exception:
            failed.append(name)
    return failed


def test_unmutated_complex_battery_passes(orc):
    assert _zbattery(orc) == []


@pytest.mark.parametrize("name,old,new", ZMUTATIONS, ids=[m[0] for m in ZMUTATIONS])
def test_planted_complex_mistake_is_caught(orc, tmp_path, name, old, new):
    with open(ZSRC) as f:
        zsrc = f.read()
    assert zsrc.count(old) == 1, f"mutation anchor not unique/not found: {name}"
    src = tmp_path / "zmutant.c"
    src.write_text(zsrc.replace(old, new))
    lib = tmp_path / "libzmutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=gnu11", "-fPIC", "-shared",
                           "-w", "-o", str(lib), SRC, str(src), "-lm"])
    with orc.using_library(str(lib)):
        failed = _zbattery(orc)
    assert failed, f"planted mistake '{name}' passed every complex pin"
