"""Pins of the angular quadrature (inputs shared by oracle and GPU path).

The S_N semi-discrete form (Section 1, eq. sntransport) needs a set with
sum_d w_d = 4 pi that integrates low-order moments exactly; the DSA
diffusion tensor (eq. SIP) is I = (1/4pi) sum_d w_d Omega Omega^T, which is
Id/3 exactly for a level-symmetric set.
"""
import math
import os

import numpy as np
import pytest

import sninputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lq_weights.txt")


def _golden():
    out = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[int(f[0])] = (float(f[1]), [float(x) for x in f[2:]])
    return out


@pytest.mark.parametrize("order", [4, 8, 12])
def test_textbook_weights(order):
    """Point weights and mu_1 agree with the tabulated LQ_N set to its 7 digits."""
    mu1, wts = _golden()[order]
    om, w = sninputs.level_symmetric(order, 3)
    assert len(w) == order * (order + 2)
    assert abs(np.min(np.abs(om)) - mu1) < 1e-7
    per_oct = w[: len(w) // 8] / (math.pi / 2)
    got = sorted(set(np.round(per_oct, 7)))
    assert np.allclose(sorted(wts), got, atol=1.5e-7)


@pytest.mark.parametrize("order,dim", [(4, 2), (8, 2), (12, 2), (4, 3), (8, 3), (12, 3)])
def test_moments(order, dim):
    om, w = sninputs.level_symmetric(order, dim)
    assert len(w) == (order * (order + 2)) // (2 if dim == 2 else 1)
    assert abs(np.sum(w) - 4 * math.pi) < 1e-13
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-14)
    # odd moments vanish, even moments of each component equal 4pi/(2n+1)
    for ax in range(3 if dim == 3 else 2):
        assert abs(np.sum(w * om[:, ax])) < 1e-13
        assert abs(np.sum(w * om[:, ax] ** 3)) < 1e-13
        for n in range(order // 2):
            assert abs(np.sum(w * om[:, ax] ** (2 * n)) - 4 * math.pi / (2 * n + 1)) < 1e-12
    # diffusion tensor I = Id/3
    I = np.einsum("d,di,dj->ij", w, om, om) / (4 * math.pi)
    assert np.allclose(I, np.eye(3) / 3, atol=1e-14)


@pytest.mark.parametrize("order", [4, 8, 12])
def test_symmetries(order):
    om, w = sninputs.level_symmetric(order, 3)
    key = {tuple(np.round(o, 12)): ww for o, ww in zip(om, w)}
    for o, ww in zip(om, w):
        # inversion (needed for L_d^T = L_{-d} pairing) and reflections
        assert abs(key[tuple(np.round(-o, 12))] - ww) < 1e-15
        for ax in range(3):
            r = o.copy()
            r[ax] = -r[ax]
            assert abs(key[tuple(np.round(r, 12))] - ww) < 1e-15
        # axis permutations
        for perm in ([1, 0, 2], [0, 2, 1], [2, 1, 0]):
            assert abs(key[tuple(np.round(o[perm], 12))] - ww) < 1e-15


def test_octant_major_order():
    om, w = sninputs.level_symmetric(8, 3)
    per = len(w) // 8
    for d in range(len(w)):
        o = (om[d, 0] < 0) + 2 * (om[d, 1] < 0) + 4 * (om[d, 2] < 0)
        assert o == d // per
    om2, w2 = sninputs.level_symmetric(8, 2)
    assert np.all(om2[:, 2] > 0)
    per2 = len(w2) // 4
    for d in range(len(w2)):
        assert (om2[d, 0] < 0) + 2 * (om2[d, 1] < 0) == d // per2


def test_config_tile_counts():
    for name, (nv, nt, nk) in {"c2": (51, 128, 77), "c3": (102, 256, 154), "c4": (51, 128, 77),
                               "c5": (102, 256, 154)}.items():
        p = sninputs.config(name)
        kind = p.meta["kind"]
        tile = p.meta["tile"]
        cells_per_tile = tile ** p.dim
        assert np.count_nonzero(kind == 0) == nv * cells_per_tile
        assert np.count_nonzero(kind == 1) == nt * cells_per_tile
        assert np.count_nonzero(kind == 2) == nk * cells_per_tile
        assert np.all(p.sigma_s <= p.sigma_t)
        assert np.all((p.q > 0) == (kind == 1))
