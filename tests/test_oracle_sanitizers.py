"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
-fsanitize=address,undefined, no recovery) runs every entry point the parity tests use on
small 2D and 3D cases -- each boundary type, k-omega transport, the tau_hat mode, the
multi-dimensional expansion, MUSCL3 and WENO5, the per-cell step, the eps and tau fields
and the per-face helpers -- with no report, and gives the same results as the default
build (which differs only in instrumentation, so the values agree to rounding order: the
sanitized build is compiled at -O1).  A host-only check: the GPU library is not involved."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent('''
    import sys
    import numpy as np
    import oracle
    from inputs import cases as C

    def cases():
        c = C.mixing_layer(12, seed=1); yield "mixing", c
        yield "sbli", C.sbli(16, 8)
        yield "iso", C.isotropic_box(6, precision="fp64")
        bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
        u = C.uniform_flow(dim=3, n=(5, 4, 3), bc=bc, vel=(0.4, 0.1, -0.2))
        rng = np.random.default_rng(3)
        u.W = u.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=u.W.shape)); yield "mixed3d", u
        s = C.shock_tube(16, 4, mu=1e-4, c_a=1.0, k_val=1e-4, omega_val=10.0); yield "sod", s
        for opt in (dict(eps_mode="tauhat"), dict(multi_d=True), dict(recon="muscl3"), dict(recon="weno5"),
                    dict(kw_transport=True), dict(kw_transport=True, recon="weno5", eps_mode="tauhat")):
            for name, base in (("ml", C.mixing_layer(10, seed=2)), ("box", C.isotropic_box(6, precision="fp64"))):
                for k, v in opt.items():
                    setattr(base, k, v)
                yield name + "+" + ",".join(opt), base

    out = []
    for name, c in cases():
        r = oracle.run_kw(c, 3) if getattr(c, "kw_transport", False) else oracle.run(c, 3)
        out.append(r["W"].ravel())
        out.append(oracle.eps_field(c, r["W"]).ravel())
        out.append(oracle.tau_field(c, r["W"]).ravel())
        if not getattr(c, "kw_transport", False):
            dt = oracle.cfl_dt(c, r["W"])
            out.append(oracle.step_cells(c, r["W"], dt, np.arange(0, c.k.size, 3)).ravel())
            out.append(oracle.strain(c, r["W"]).ravel())
            out.append(oracle.ghost_fill(c, r["W"]).ravel())
    out.append(np.ravel(oracle.kogan(0.3, 1.0)))
    out.append(np.ravel(oracle.kogan_e(0.3, 0.1, 1.0)))
    out.append(np.ravel(oracle.moments_u(0.4, 2.0)))
    np.save(sys.argv[1], np.concatenate(out))
    print("driver done", flush=True)
''')


def _build_sanitized(path, src=None):
    src = src or os.path.join(ROOT, "oracle", "gks_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", path, src, "-lm"]
    subprocess.check_call(cmd)


def _run(lib_path, out, env_extra):
    code = ("import oracle\n"
            + (f"oracle.use_library({lib_path!r})\n" if lib_path else "")
            + DRIVER)
    env = dict(os.environ, OMP_NUM_THREADS="2", PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""),
               **env_extra)
    return subprocess.run([sys.executable, "-c", code, out], cwd=ROOT, capture_output=True, text=True,
                          timeout=900, env=env)


def test_oracle_under_asan_and_ubsan(tmp_path):
    import numpy as np
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libgks_oracle_san.so")
    _build_sanitized(lib)
    san_env = {"LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
               "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    r = _run(lib, str(tmp_path / "san.npy"), san_env)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "driver done" in r.stdout, report
    for marker in ("AddressSanitizer", "runtime error", "LeakSanitizer"):
        assert marker not in r.stderr, report
    r0 = _run(None, str(tmp_path / "ref.npy"), {})
    assert r0.returncode == 0, r0.stderr[-4000:]
    a, b = np.load(tmp_path / "san.npy"), np.load(tmp_path / "ref.npy")
    assert a.shape == b.shape
    scale = np.maximum(np.abs(b), 1e-300)
    assert np.all(np.abs(a - b) <= 1e-11 * np.maximum(scale, np.max(np.abs(b)) * 1e-6)), np.max(np.abs(a - b))


def test_the_sanitized_build_catches_a_planted_overflow(tmp_path):
    """The instrumentation is live: a copy of the oracle whose moment-system matrix is one
    column short (3D indexes past the row's end) is stopped, by UBSan's bounds check at
    compile-time-known array sizes, else by AddressSanitizer at the stack array's end."""
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    text = open(os.path.join(ROOT, "oracle", "gks_oracle.c")).read()
    assert text.count("double A[5][6];") == 1
    src = tmp_path / "planted.c"
    src.write_text(text.replace("double A[5][6];", "double A[5][5];"))
    lib = str(tmp_path / "libplanted.so")
    _build_sanitized(lib, str(src))
    r = _run(lib, str(tmp_path / "p.npy"), {"LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1"})
    assert r.returncode != 0
    assert "out of bounds" in r.stderr or "stack-buffer-overflow" in r.stderr, r.stderr[-3000:]
