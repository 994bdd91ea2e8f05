"""Each planted mistake in the oracle (ORACLE_MUTANT=k in oracle.cpp) must be
caught by at least one pin.  Mutants are built with g++ into a temporary
directory; nothing here touches a GPU."""
import os

import pytest

from oracle import Oracle
from oracle.build import build
from oracle_pins import all_pins

MUTANTS = {
    1: "drops the last product of every B row",
    2: "walks B's row i instead of row k",
    3: "(min,+) takes the max",
    4: "float64 sum overwrites instead of accumulating",
    5: "skips the first stored entry of each A row",
    6: "|product| sums use the signed value",
    7: "merge forgets the last part",
    8: "int64 products truncated to 32 bits",
    9: "(max,x) takes the min",
    10: "(min,max) multiplies by the min",
}


@pytest.mark.parametrize("k", sorted(MUTANTS), ids=[f"mutant{k}" for k in sorted(MUTANTS)])
def test_mutant_is_caught(tmp_path, k):
    path = build(mutant=k, out=os.path.join(str(tmp_path), f"liboracle_m{k}.so"))
    orc = Oracle(path)
    caught = []
    for name, fn in all_pins():
        try:
            fn(orc)
        except AssertionError:
            caught.append(name)
        except Exception as e:  # a crash of the mutant also counts as caught
            caught.append(f"{name}:{type(e).__name__}")
        if caught:
            break
    assert caught, f"no pin caught mutant {k} ({MUTANTS[k]})"


# planted mistakes in the Python parts of the oracle (module switch MUTANT)
PY_MUTANTS = {
    ("power", 1): "linear powers multiply by the current power instead of W'",
    ("power", 2): "self loops are never merged in",
    ("power", 3): "the fixed-point test ignores the values",
    ("dcsc", 4): "decompression counts the column itself as before it",
    ("dcsc", 5): "compression drops the last non-empty column",
    ("dcsc", 6): "the CSC product multiplies in the wrong order",
}


@pytest.mark.parametrize("mod,k", sorted(PY_MUTANTS), ids=[f"{m}{k}" for m, k in sorted(PY_MUTANTS)])
def test_python_mutant_is_caught(orc, mod, k):
    import importlib
    m = importlib.import_module(f"oracle.{mod}")
    caught = []
    m.MUTANT = k
    try:
        for name, fn in all_pins():
            try:
                fn(orc)
            except AssertionError:
                caught.append(name)
            except Exception as e:
                caught.append(f"{name}:{type(e).__name__}")
            if caught:
                break
    finally:
        m.MUTANT = 0
    assert caught, f"no pin caught {mod} mutant {k} ({PY_MUTANTS[(mod, k)]})"
