"""sn_response_noalloc (fixed device scratch, no allocation) against
sn_response through the C ABI: two calls in a row, the second on a smaller
problem, each bit-for-bit equal to sn_response; a third call on the first
problem again (the scratch keeps nothing between calls that matters); and the
rejection of a quadrature too large for the fixed scratch."""
import math

import numpy as np
import pytest

import sninputs
from gpu_util import context, dev, random_problem, say
from sninputs import Problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(p, seed, prec):
    from paper_2001_09196_amd import sn_response, sn_response_noalloc, sn_sweep
    rng = np.random.default_rng(seed)
    phi = dev(rng.uniform(0, 1, (p.ncells, p.nn)))
    r = dev(rng.uniform(0, 2, p.ncells))
    face = 2 * p.dim - 1
    dt = torch.float64 if prec == 0 else torch.float32
    with context(p) as ctx:
        psi = torch.empty((p.ncells, p.ndirs, p.nn), dtype=dt, device="cuda")
        sn_sweep(ctx, phi, dev(p.q), None, False, prec, psi)
        got = [sn_response_noalloc(ctx, r, phi, face, psi, prec), sn_response_noalloc(ctx, None, None, face, psi, prec),
               sn_response_noalloc(ctx, r, phi, -1, None, prec)]
        ref = [sn_response(ctx, r, phi, face, psi, prec), sn_response(ctx, None, None, face, psi, prec),
               sn_response(ctx, r, phi, -1, None, prec)]
    say(f"  {p.name}: {got[0]:.17g} vs {ref[0]:.17g}")
    return got, ref


def test_noalloc_matches_response_twice_then_smaller():
    big = random_problem(3, 21, 13, 9, order=8, seed=3)       # 2457 cells, 80 dirs
    small = random_problem(2, 9, 7, 1, order=4, seed=4)        # 63 cells, 12 dirs
    say("no-alloc response: large, small, large")
    for p, seed, prec in ((big, 5, 0), (small, 6, 1), (big, 5, 0)):
        got, ref = _case(p, seed, prec)
        assert got == ref
        assert all(math.isfinite(v) for v in got)


def test_noalloc_rejects_oversize_quadrature():
    from paper_2001_09196_amd import SnError, sn_response_noalloc
    from paper_2001_09196_amd.binding import SN_ERR_INVALID
    n = 16400                                                   # > 16384 - 3 * 1 - 3 on this mesh
    rng = np.random.default_rng(7)
    om = rng.standard_normal((n, 3))
    om /= np.linalg.norm(om, axis=1)[:, None]
    w = np.full(n, 4 * math.pi / n)
    w[-1] = 4 * math.pi - np.sum(w[:-1])                        # the sum is 4 pi to rounding
    p = Problem("many", 2, 3, 3, 1, (1.0, 1.0, 1.0), np.ones(9), np.full(9, 0.5), np.ones(9), om, w)
    with context(p) as ctx:
        phi = dev(np.ones((9, 4)))
        with pytest.raises(SnError) as e:
            sn_response_noalloc(ctx, dev(np.ones(9)), phi, -1, None, 0)
        assert e.value.code == SN_ERR_INVALID
        assert "scratch" in str(e.value)
