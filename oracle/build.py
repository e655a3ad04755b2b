"""Compile the CPU reference library (test infrastructure; see smc2_oracle.h)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_smc2.so")


def build_oracle(verbose: bool = False, src_dir: str = HERE, out: str = LIB) -> str:
    """Build smc2_oracle.c from src_dir (default: this directory) into out. Tests build
    copies with a planted mistake from another directory the same way."""
    # -ffp-contract=off: every float/double operation is rounded on its own, which
    # is what the precision conventions of the reference state.
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           os.path.join(src_dir, "smc2_oracle.c"), "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose=True))
