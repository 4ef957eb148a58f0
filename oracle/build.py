"""Build step for the reference library (test infrastructure; see lbm_oracle.cpp)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
# LBM_ORACLE_LIB points the loader at another build of the reference (the mutation tests load planted copies)
LIB = os.environ.get("LBM_ORACLE_LIB") or os.path.join(HERE, "liblbm_oracle.so")


def build(force: bool = True) -> str:
    """Compile lbm_oracle.cpp into liblbm_oracle.so with g++ (-O2, OpenMP). Returns the library path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
