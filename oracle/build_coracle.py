"""Build the C oracle (test infrastructure) into oracle/libcoracle.so with gcc + OpenMP."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    src = os.path.join(HERE, "coracle.c")
    out = os.path.join(HERE, "libcoracle.so")
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", src, "-o", out + ".tmp", "-lm"]
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build()
