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
