"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host C code
(CPU only): the oracle and the quadruple-precision reference are compiled
with -fsanitize=address,undefined (errors fatal) and exercised in a child
process with the sanitizer runtime preloaded: Algorithms 1-3 on stencil,
CSR, dense and low-rank operators (and over C on complex dense and CSR ones), ragged sizes, p = 0 and p = 7, the single
block series, the integrator and the error paths (bad arguments, term cap,
overflow guard).  Any out-of-bounds access, use after free or undefined
operation aborts the child, and the test fails with its report."""
import os
import subprocess
import sys
import tempfile
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r"""
    import sys
    import numpy as np
    sys.path.insert(0, sys.argv[1])
    sys.path.insert(0, sys.argv[1] + "/tests")
    import oracle
    import refs
    import workloads as wl
    import ctypes
    ctypes.CDLL(None)["__asan_init"]          # the sanitizer runtime is loaded
    oracle._lib = oracle._configure(ctypes.CDLL(sys.argv[2]))
    assert oracle._lib["__ubsan_handle_add_overflow_abort"] is not None
    refs._EXACT_Q = None
    probs = [wl.config1(), wl.config2(nside=13), wl.config3(nside=6, nonnormal=True, tol=1e-8),
             wl.small_problem(9, 7, 3, seed=1), wl.small_problem(5, 0, 2, seed=2),
             wl.exp3_problem("M2", 1.0, n=301), wl.exp2_problems(N=12)[1]]
    for pr in probs:
        W, st, prm = oracle.full(pr)
        assert np.isfinite(W).all(), pr.name
        oracle.series_block(pr.op, pr.p, pr.r, pr.t * 0.01, pr.beta, pr.V, pr.tol)
    op = wl.adr_operator(6)
    po = oracle.params(op, 1e-7, wl.params_vector(op.n))
    oracle.exprk4s6(op, wl.adr_reaction(20.0), wl.adr_initial(6), 1e-3, 3, 1e-7,
                    po["shift"], po["s"])
    pr = wl.config2(nside=9)
    for bad in ([np.nan, 1e-4, 1e-4], [1e300, 1.0, 1.0]):
        try:
            oracle.solve(pr.op, 3, 3, bad, pr.beta, pr.V, 1e-12, 0.0, 1e5)
        except oracle.OracleError:
            pass
    try:
        oracle.solve(pr.op, 3, 3, pr.t, pr.beta, pr.V, 1e-12, 0.0, 1e5, kcap=3)
    except oracle.OracleError:
        pass
    big = wl.CSR(4, np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32), np.full(4, 1e300))
    try:
        oracle.params(big, 1e-8, np.ones(4))
    except oracle.OracleError:
        pass
    pq = wl.small_problem(4, 2, 1, seed=3)
    refs.exact_dense_q(pq.op.A, pq.t, pq.beta, pq.V)
    # the complex algorithms: dense and CSR, p = 0 and p = 5, error paths
    rng = np.random.default_rng(4)
    for n, p, r in ((7, 5, 3), (3, 0, 1)):
        Az = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) - 3.0 * np.eye(n)
        zop = oracle.ZOperator(dense=Az)
        zp = oracle.zparams(zop, 2.0 ** -53, np.ones(n))
        tz = np.exp(1j * np.arange(r)) * 4.0
        Vz = rng.standard_normal((n, p + 1)) + 1j * rng.standard_normal((n, p + 1))
        oracle.zsolve(zop, p, r, tz, np.ones((r, p + 1)), Vz, 1e-12, zp["shift"] + 1j, zp["s"])
        oracle.zsolve(zop, p, r, tz, None, Vz, 1e-12, zp["shift"], zp["s"], form="alpha",
                      alpha=np.ones(r) * 1j)
    zc = oracle.ZOperator(csr=(np.arange(5), np.arange(4), np.full(4, 1e300 + 0j)))
    try:
        oracle.zparams(zc, 1e-8, np.ones(4))
    except oracle.OracleError:
        pass
    try:
        oracle.zsolve(zc, 1, 1, [np.nan], np.ones((1, 2)), np.ones((4, 2)), 1e-8, 0.0, 1.0)
    except oracle.OracleError:
        pass
    print("SANITIZED_OK")
""")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc here")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-std=gnu11",
             "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    lib = str(tmp_path / "liborc_asan.so")
    subprocess.check_call(["gcc"] + flags + ["-o", lib,
                                             os.path.join(ROOT, "oracle", "phicomb_oracle.c"),
                                             os.path.join(ROOT, "oracle",
                                                          "phicomb_oracle_complex.c"),
                                             "-lm"])
    # the quadruple-precision reference, sanitized too, where refs looks for it
    qlib = str(tmp_path / "libexact_q.so")
    subprocess.check_call(["gcc"] + flags + ["-o", qlib,
                                             os.path.join(ROOT, "tests", "exact_q.c"),
                                             "-lquadmath", "-lm"])
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + ((" " + _runtime("libubsan.so")) if _runtime("libubsan.so") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PHICOMB_EXACT_Q_LIB"] = qlib
    p = subprocess.run([sys.executable, str(script), ROOT, lib], capture_output=True, text=True,
                       env=env, timeout=600)
    assert p.returncode == 0 and "SANITIZED_OK" in p.stdout, (p.stdout[-3000:], p.stderr[-6000:])
