"""Every planted mistake in the oracle fails at least one of its pins.

Altered copies of oracle/mh_oracle.c (one mistake each, listed in
oracle_mutants.py) are compiled with the oracle's own flags and their pins are
run against them in child processes; the unaltered source must pass the same
pins.  This shows that the pins constrain the oracle's arithmetic rather than
only its own restatement of it.
"""
import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
import oracle_mutants as om

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "mh_oracle.c")


def _build(src_text: str, path: str) -> None:
    c = path[:-3] + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    inc = os.path.join(os.path.dirname(HERE), "oracle")
    subprocess.run(["gcc", *oracle.CFLAGS, "-I", inc, "-o", path, c, "-lm"], check=True)


def _pins(lib_path: str, name: str) -> dict:
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_mutants.py"), lib_path, name],
                       capture_output=True, text=True, timeout=300)
    last = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not last:
        # a mutant that crashes its pins has been caught as well
        return {"(child)": f"fail: exit {r.returncode}: {r.stderr.strip().splitlines()[-1:]}"}
    return json.loads(last[-1])


def test_pristine_oracle_passes_every_mutant_pin(tmp_path):
    with open(SRC) as f:
        text = f.read()
    lib = str(tmp_path / "liboracle_pristine.so")
    _build(text, lib)
    res = _pins(lib, "*")
    assert res and all(v == "pass" for v in res.values()), res


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with open(SRC) as f:
        text = f.read()

    def one(k):
        name, old, new, occ, _ = om.MUTANTS[k]
        lib = str(tmp_path / f"liboracle_m{k}.so")
        _build(om.mutate(text, old, new, occ), lib)
        return name, _pins(lib, name)

    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(one, range(len(om.MUTANTS))))
    survivors = {name: res for name, res in results if all(v == "pass" for v in res.values())}
    assert not survivors, survivors
    # each mutant is caught by a failing pin, not by a build problem
    assert all(any(v.startswith("fail") for v in res.values()) for _, res in results)


@pytest.mark.parametrize("k", range(len(om.MUTANTS)))
def test_mutation_text_is_present(k):
    # the replaced text exists exactly where the mutant expects it
    with open(SRC) as f:
        text = f.read()
    name, old, new, occ, _ = om.MUTANTS[k]
    assert om.mutate(text, old, new, occ) != text, name
