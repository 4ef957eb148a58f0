"""The reference's pins catch plausible mistakes: each case plants one mistake in a copy of the reference source
(compiled on the CPU into a temporary library) and runs the pins that cover that part against it; they must fail.
The unmodified source passes the same pins (the rest of the suite)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.cpp")

# (name, text in the reference, planted replacement, pin tests that must catch it)
MUTATIONS = [
    ("tanh_factor", "std::tanh(2.0 * (dist - R[d]) / W)", "std::tanh((dist - R[d]) / W)",
     "tests/test_oracle_force_init.py"),
    ("no_nearest_image_x", "dx -= p->nx * std::floor(dx / p->nx + 0.5);", "",
     "tests/test_oracle_force_init.py"),
    ("sum_not_max", "if (v > r) r = v;", "r += v - rho_v;", "tests/test_oracle_force_init.py"),
    ("swap_A_and_1_minus_A",
     "*Fx = -p.A * su_x - (1.0 - p.A) * G_f * pc * sp_x;\n    *Fy = -p.A * su_y - (1.0 - p.A) * G_f * pc * sp_y;",
     "*Fx = -(1.0 - p.A) * su_x - p.A * G_f * pc * sp_x;\n    *Fy = -(1.0 - p.A) * su_y - p.A * G_f * pc * sp_y;",
     "tests/test_oracle_force_init.py"),
    ("potential_without_half", "S U = G_f * pn * pn / 2.0;", "S U = G_f * pn * pn;",
     "tests/test_oracle_force_init.py"),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_its_pins(tmp_path, name, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found once"
    mutated = tmp_path / "lbm_oracle_mutant.cpp"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liblbm_oracle_mutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-fopenmp", str(mutated), "-o", str(lib)],
                   check=True)
    env = dict(os.environ, LBM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", pins],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 1, f"planted {name} was not caught:\n{res.stdout[-2000:]}"
    assert "failed" in res.stdout


def test_unmodified_copy_passes_the_same_pins(tmp_path):
    """Control: the same build and loading path with the source unchanged passes."""
    lib = tmp_path / "liblbm_oracle_copy.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-fopenmp", SRC, "-o", str(lib)], check=True)
    env = dict(os.environ, LBM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          "tests/test_oracle_force_init.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0, res.stdout[-2000:]
