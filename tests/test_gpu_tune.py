"""The autotuner through the C ABI: the settings it picks run, pass the
accuracy gate against the oracle, and are written into every instance of a
group."""
import sys

import numpy as np
import pytest

from conftest import rel
from paper_2004_00546_amd import _lib, api, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    _lib.load()
    return _t


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_autotune_linear_1d(torch, orc):
    inst = workloads.make("advdiff1d_n128")[0]
    probs, rep = api.autotune([inst], p_min=2, p_max=50, rtol=1e-9, krylov="poly")
    r = rep[0]
    say("tuned C1:", r)
    assert r["rel_err"] >= 0 and r["rel_err"] <= 1e-9
    assert r["ms"] > 0 and r["serial_ms"] > 0 and r["candidates"] > 1
    assert probs[0].P == r["P"] and inst["n_steps"] % probs[0].P == 0
    run = api.GradientRunner([inst], problems=probs)
    run.run()
    assert run.status()[0] == 0
    got = run.results()[0]
    assert rel(got["grad"], orc.gradient(inst)["grad"]) < 1e-8


def test_autotune_burgers_group(torch, orc):
    """Three Burgers instances of one grid form one group: the longest is
    timed, the others get P with the same steps per slice."""
    base = workloads.make("burgers1d_ragged")
    picks = [i for i in range(len(base)) if base[i]["nx"] == 1024][:3]
    insts = []
    for i in picks:
        nt = base[i]["n_steps"] // 4
        insts.append(dict(base[i], n_steps=nt, T=base[i]["T"] / 4, P=base[i]["P"] // 4))
    probs, rep = api.autotune(insts, p_min=8, p_max=128, rtol=1e-9)
    say("tuned burgers group:", rep)
    assert len({r["group"] for r in rep}) == 1
    for inst, p, r in zip(insts, probs, rep):
        assert inst["n_steps"] % p.P == 0
        assert p.krylov == rep[0]["krylov"]
    run = api.GradientRunner(insts, problems=probs)
    run.run()
    assert run.status()[0] == 0
    for inst, got in zip(insts, run.results()):
        e = rel(got["grad"], orc.gradient(inst)["grad"])
        say("  n_steps %d P %d grad %.2e" % (inst["n_steps"], probs[insts.index(inst)].P, e))
        assert e < 1e-8
