"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only), driven through its ctypes binding over the paths the pins
use: spline evaluation, wrap, cell ids, cell and brute-force lists (periodic,
orthorhombic and open boxes), forces, the velocity-Verlet loop with rebuilds,
the closed-form potential, the force-matching loss and gradient, and the
multi-species forms.  Any out-of-bounds access, use after free or undefined
operation ends the child process with an error report."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle
    oracle._LIB = {lib!r}
    from workloads import configs, potential as P

    oracle.set_threads(1)
    tabs = P.md_tables()
    oracle.spline_eval(tabs[2], np.linspace(-1.0, 45.0, 101))
    kw = dict(mass=configs.MASS, dt=configs.DT, r_cut=P.RC, skin=configs.SKIN,
              ftm2v=configs.FTM2V)
    boxes = [configs.small_box(5, seed=1, temperature=3000.0, sigma_x=0.1),
             configs.ortho_box(5, 6, 7, seed=2, temperature=2000.0),
             configs.slab(5, 5, 5, seed=3, sigma_x=0.05, vacuum=6.0)]
    for b in boxes:
        oracle.cell_ids(b.x, b.box, P.RC + configs.SKIN)
        for method in ("cells", "brute"):
            oracle.neighbor_list(b.x, b.box, P.RC + configs.SKIN, cap=128, method=method)
        oracle.forces_at(b.x, b.box, tabs, P.RC, configs.SKIN)
        out = oracle.md_run(b.x, b.v, b.box, tabs, 30, want_energy=True, **kw)
        assert out["code"] == 0, out["code"]
    b = boxes[0]
    oracle.forces_analytic(b.x, b.box, P.analytic_params())
    fb = configs.config_fm(3, 5)
    x = np.concatenate([c.x for c in fb])
    off = np.concatenate([[0], np.cumsum([c.n for c in fb])])
    fref = np.concatenate([oracle.forces_analytic(c.x, c.box, P.analytic_params())[0] for c in fb])
    oracle.fm_loss_grad(x, off, np.stack([c.box for c in fb]), P.fm_tables(), fref)
    a = configs.alloy_box(5, seed=4)
    oracle.forces_at_multi(a.x, a.box, a.types, P.alloy_tables(), P.RC, configs.SKIN)
    out = oracle.md_run_multi(a.x, a.v, a.box, a.types, P.alloy_tables(), P.ALLOY_MASS, 20,
                              dt=configs.DT, r_cut=P.RC, skin=configs.SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0, out["code"]
    print("SANITIZED_OK")
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas", "-o", lib,
           os.path.join(ROOT, "oracle", "eam_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join(p for p in (asan, env.get("LD_PRELOAD", "")) if p)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=600)
    report = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
