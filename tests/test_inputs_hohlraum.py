"""The pseudo-scattering TRT inputs (Sec. 4.2, eqs. hohlraum_sigma and
hohlraum_q) and the synthetic hohlraum layout."""
import math

import numpy as np

import sninputs


def test_trt_closed_forms_and_limits():
    a, c = sninputs.TRT_A, sninputs.TRT_C
    for sigma, cv, T, dt in ((1e3, 1e5, 0.4, 1e-3), (1.0, 1.0, 1e-3, 1e-3), (100.0, 1e3, 0.05, 0.1)):
        sps, qps = sninputs.trt_pseudo_scattering(sigma, cv, T, dt)
        x = sigma * 16 * math.pi * a * c * T ** 3 * dt / cv          # coupling of one step
        assert math.isclose(float(sps), sigma * x / (1 + x), rel_tol=1e-12)
        assert math.isclose(float(qps), sigma * a * c * T ** 4 / (1 + x), rel_tol=1e-9)
        assert 0 < sps < sigma and qps > 0
    # no heat capacity: all absorption is re-emitted (pure scatterer, no source);
    # infinite heat capacity: no scattering, equilibrium emission sigma a c T^4
    s0, q0 = sninputs.trt_pseudo_scattering(50.0, 1e-30, 0.3, 1.0)
    assert math.isclose(float(s0), 50.0, rel_tol=1e-12) and abs(float(q0)) <= 1e-9 * 50 * a * c * 0.3 ** 4
    s1, q1 = sninputs.trt_pseudo_scattering(50.0, 1e30, 0.3, 1.0)
    assert float(s1) < 1e-15 and math.isclose(float(q1), 50 * a * c * 0.3 ** 4, rel_tol=1e-12)


def test_hohlraum_layout():
    nx, ny = 80, 40
    p = sninputs.hohlraum(nx, ny, sn=4, order=3)
    reg = p.meta["regions"].reshape(ny, nx)
    assert np.array_equal(reg, reg[:, ::-1]) and np.array_equal(reg, reg[::-1, :])   # symmetric
    names = sninputs.HOHLRAUM_REGIONS

    def runs(row):
        out = [names[row[0]]]
        for k in row[1:]:
            if names[k] != out[-1]:
                out.append(names[k])
        return out
    assert runs(reg[ny // 2]) == ["helium", "ch", "hydrogen", "ch", "helium"]          # through the holes
    assert runs(reg[int(0.26 * ny)]) == ["gold", "helium", "ch", "helium", "gold"]          # below the holes
    thick = p.sigma_s >= 1.0
    assert 0.02 <= thick.mean() <= 0.035                      # the paper's 2.3-2.9% thick DOFs
    assert np.all(reg.ravel()[thick] == 1)                    # only the heated gold is thick
    assert np.all(p.sigma_s <= p.sigma_t) and np.all(p.q > 0)
    hot = reg.ravel() == 1
    assert p.q[hot].min() > 1e4 * p.q[~hot].max()              # the laser-heated wall is the source
    assert p.nn == 16 and p.ndirs == 12
