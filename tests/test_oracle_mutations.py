"""Planted mistakes in the oracle, on the CPU: each entry of
``oracle_mutations.MUTATIONS`` is applied to a copy of ``oracle/lbm_oracle.c``,
compiled, and the pins named with it are run against that build (through the
``LBM_ORACLE_LIB`` override of the oracle package).  Every mutant must fail
them: a pin set that a plausible mistake passes pins nothing.  The unmutated
oracle passes the same pins in ``test_oracle_pins.py``."""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

import oracle as O

from oracle_mutations import MUTATIONS

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINS = os.path.join(HERE, "test_oracle_pins.py")


def _check(m, workdir, src):
    name, old, new, count, select = m
    if src.count(old) != count:
        return name, f"the text to change occurs {src.count(old)} times, expected {count}"
    d = os.path.join(workdir, name)
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "lbm_oracle.c"), "w") as fh:
        fh.write(src.replace(old, new))
    lib = O.compile_oracle(os.path.join(d, "lbm_oracle.c"), os.path.join(d, "liblbm_oracle.so"))
    env = dict(os.environ, LBM_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        PINS, "-k", select], capture_output=True, text=True, env=env, cwd=ROOT)
    if r.returncode == 1:  # at least one selected pin failed
        return name, None
    if r.returncode == 5:
        return name, f"no pin matches -k {select!r}"
    return name, f"pins {select!r} did not catch it (pytest rc {r.returncode})"


def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = open(os.path.join(ROOT, "oracle", "lbm_oracle.c")).read()
    O.build(force=False)  # the header the copies include is the repository's
    workers = max(1, min(8, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda m: _check(m, str(tmp_path), src), MUTATIONS))
    bad = [(n, msg) for n, msg in res if msg]
    assert not bad, bad
    assert len(res) == len(MUTATIONS) >= 30


@pytest.mark.parametrize("name", ["sa_fw_exponent", "sa_fv2_dropped", "sa_r_zero_when_s_tilde_negative"])
def test_sa_near_wall_mistakes_are_listed(name):
    """The three Spalart-Allmaras mistakes that used to pass every pin are in
    the planted set."""
    assert name in {m[0] for m in MUTATIONS}
