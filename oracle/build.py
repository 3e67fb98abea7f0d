"""Compile the plain-C oracle with gcc (no GPU code)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(HERE, "_build", "liboracle_hv.so")


def build_oracle(verbose: bool = False) -> str:
    out = library_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    src = os.path.join(HERE, "c", "hv_bsearch.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", out + ".tmp", src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + res.stderr)
    os.replace(out + ".tmp", out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build_oracle(verbose=True)
