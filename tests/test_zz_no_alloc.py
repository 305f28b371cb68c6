"""GPU test of the allocation-free entry point cmcg_apply_static: its results equal those of
cmcg_apply through a handle, bit for bit, for every operator and both precisions, on two calls
in a row (the second on a smaller problem, in the buffer the first call left behind), and a
problem larger than its fixed buffer is refused before any device work."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f1 import F1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _problem(nx, ny, seed, masked=False):
    """Ragged grid, random c, complex source, data on two absorbing faces, one Neumann face;
    optionally a block of Dirichlet cells with data."""
    rng = np.random.default_rng(seed)
    c = 1.0 + rng.uniform(size=(ny, nx))
    f = np.zeros((ny, nx), complex)
    f[5:9, 10:14] = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    gS = [rng.standard_normal(ny) + 1j * rng.standard_normal(ny), np.zeros(ny, complex),
          rng.standard_normal(nx) + 1j * rng.standard_normal(nx), np.zeros(nx, complex)]
    mask = gD = None
    if masked:
        mask = np.zeros((ny, nx), np.uint8)
        mask[ny // 3: ny // 3 + 6, nx // 2: nx // 2 + 9] = 1
        gD = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=2 * math.pi * 2.5, c=c, f=f, gS=gS,
                   sound_soft=mask, gD=gD, face_bc=(0, 0, 0, 1), courant=0.5, name="static")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_apply_equals_handle_apply(cm, prec):
    import torch
    ops = (cm.OP_FORWARD, cm.OP_FORCED, cm.OP_ADJOINT, cm.OP_RIESZ)
    # two calls in a row on the same buffer, the second problem smaller than the first
    for nx, ny, seed, masked in ((300, 260, 3, True), (70, 37, 5, False)):
        prob = _problem(nx, ny, seed, masked)
        with cm.Solver(prob, prec) as s:
            n = s.info["state_len"]
            g = torch.Generator(device="cuda").manual_seed(seed)
            z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
            ref = {op: s.apply(op, z) for op in ops}
            part = s.apply(cm.OP_FORCED, z, steps=5)
        for op in ops:
            got = cm.apply_static(prob, op, z, precision=prec)
            assert torch.equal(got, ref[op]), (nx, op)
        assert torch.equal(cm.apply_static(prob, cm.OP_FORCED, z, precision=prec, steps=5), part)
        # in place, as cmcg_apply allows
        zz = z.clone()
        cm.apply_static(prob, cm.OP_ADJOINT, zz, precision=prec, out=zz)
        assert torch.equal(zz, ref[cm.OP_ADJOINT])
        if prec == "fp64" and not masked:
            o = F1(prob)
            zn = z.cpu().numpy()
            assert np.linalg.norm(ref[cm.OP_FORCED].cpu().numpy() - o.period(zn, True)) <= \
                1e-13 * np.linalg.norm(o.period(zn, True))


def test_static_apply_refuses_a_problem_beyond_its_buffer(cm):
    import torch
    prob = ci.random_medium_2d(n=1024, freq=10.0, n_src=1, seed=2)
    n = 1024 * 1023 * 2 + 1024 * 1024
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CMCGError) as e:
        cm.apply_static(prob, cm.OP_FORWARD, z)
    assert e.value.status == cm.ENOMEM and "MiB" in str(e.value)
