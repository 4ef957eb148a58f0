"""The reference library built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, g++) and run through
every option: walls with a different angle per column, the piecewise-linear EOS with the surface-tension source,
Martys-Chen walls with MRT rates, periodic rows, Eq. 19 with the plain Shan-Chen force, the complex-step path, and
the EOS solvers. Any out-of-bounds access, use of uninitialised memory caught by the runtimes, or undefined
behaviour aborts the child process."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def runtime(name):
    path = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_reference_runs_clean_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liblbm_oracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "lbm_oracle.cpp"), "-o", lib], check=True)
    script = textwrap.dedent(f"""
        import math, sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        from oracle import build as B
        B.LIB = {lib!r}
        from oracle import oracle as ora
        PW10 = (0.25, -0.02, 0.3, 1.0, 10.0)
        for T, kw in [(0.85, {{}}), (1.0, dict(piecewise=PW10, kappa=0.5)),
                      (0.75, dict(G_w=(-0.3, -0.2), mrt=(1.2, 1.4, 1.1))),
                      (0.85, dict(periodic_y=True, kappa=0.3, tau=0.8)), (0.85, dict(wet_iters=0, A=0.0))]:
            nx, ny = 33, 12
            s = ora.Sim(nx, ny, T, theta_bottom=np.radians(np.linspace(40, 140, nx)), theta_top=math.radians(100.0),
                        **kw)
            s.init_droplets([16.0], [0.5 if not kw.get("periodic_y") else 6.0], [6.0])
            s.run(20)
            fc = s.run_cplx(2, s.f + 1e-30j, s.theta_b, s.theta_t, -1.0 + 1e-30j, -1.0)
            r, p = s.density()
            assert np.isfinite(r).all() and np.isfinite(fc).all()
            ora.collide_mrt_node(ora.Sim(4, 4, 0.7, mrt=(1.1, 1.2, 1.3), kappa=0.5), r[5, :9], 1e-4, -1e-4,
                                 (1e-3, 2e-3, 3e-4))
        ora.pw_breakpoints(*PW10)
        ora.cs_maxwell(ora.cs_critical()[1] * 0.7)
        ora.ghost_density(0.1, 0.2, 0.15, 0.2, 0.3, 4)
        print("sanitized run complete")
    """)
    env = dict(os.environ, LD_PRELOAD=runtime("libasan.so"), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "sanitized run complete" in res.stdout, res.stderr[-4000:]
