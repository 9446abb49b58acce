"""Argument checks of the autograd interface (host side, no GPU): an MGRIT
forward whose parameters do not describe the differentiated solve is refused
before any device work, and the caller's parameters are left untouched."""
import pytest
import torch

from paper_2104_09404_amd import autograd as AG
from paper_2104_09404_amd import mgrit as M

NX, NT, DT = 64, 32, 1e-3


def run(p, nt=NT, dt=DT, u0=None, every=8, solver="mgrit"):
    u0 = torch.zeros(NX, dtype=torch.float64) if u0 is None else u0
    return AG.solve(u0, M.scheme(NX), dt, nt, every=every, solver=solver, mgrit_params=p)


@pytest.mark.parametrize("change,match", [
    (dict(nt=64), "nt"),
    (dict(dt=2e-3), "dt"),
    (dict(init=1), "init"),
    (dict(m=3), "multiple"),
])
def test_mismatched_mgrit_parameters_are_refused(change, match):
    kw = dict(nt=NT, dt=DT, m=4, levels=2)
    kw.update({k: v for k, v in change.items() if k in ("nt", "dt", "m")})
    p = M.params(kw["nt"], kw["dt"], kw["m"], kw["levels"], init=change.get("init", 0))
    with pytest.raises(ValueError, match=match):
        run(p)
    assert p.storage == 0


def test_missing_parameters_and_bad_inputs_are_refused():
    with pytest.raises(ValueError, match="needs mgrit parameters"):
        run(None)
    with pytest.raises(ValueError, match="nx"):
        run(M.params(NT, DT, 4, 2), u0=torch.zeros(NX + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="nx"):
        run(M.params(NT, DT, 4, 2), u0=torch.zeros(NX, dtype=torch.float32))
    with pytest.raises(ValueError, match="checkpoint spacing"):
        run(None, every=5, solver="serial")


def test_parameter_copy_keeps_caller_storage():
    p = M.params(NT, DT, 4, 2, storage=0)
    q = AG._mgrit_forward_params(p, NT, DT)
    assert q.storage == 1 and p.storage == 0
    assert (q.nt, q.m, q.levels, q.dt) == (p.nt, p.m, p.levels, p.dt)
