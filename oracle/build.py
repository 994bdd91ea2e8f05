"""Build ``oracle/liboracle.so`` (g++, OpenMP, no FP contraction).

``build(mutant=k, out=path)`` builds a variant with deliberate mistake k
planted (see ``oracle.cpp``), used only by the oracle's own pin tests.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(mutant: int = 0, out: str = None, verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.cpp")
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
           f"-DORACLE_MUTANT={int(mutant)}", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
