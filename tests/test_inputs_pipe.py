"""The synthetic crooked-pipe inputs (Sec. 4.1 stand-in): region shares that
reproduce the thin/thick percentages of the paper's five problems at
eta = 1 (Table problems), sigma_t = sigma_s + 1/(c dt), and the source."""
import numpy as np
import pytest

import sninputs

# thin/thick percentages printed for problems #1..#5 at eta = 1 (Table problems)
PAPER_THICK = {1: 0.45, 2: 0.68, 3: 0.61, 4: 0.32, 5: 0.68}


@pytest.mark.parametrize("k", sorted(PAPER_THICK))
def test_thick_shares_match_table(k):
    p = sninputs.crooked_pipe(k, 1e3)
    assert abs(p.thick_mask(1.0).mean() - PAPER_THICK[k]) <= 0.015


def test_cross_sections_and_source():
    p = sninputs.crooked_pipe(2, 1e3, cells_per_unit=4)
    reg = p.meta["regions"]
    assert p.nx == 56 and p.ny == 40 and p.h[0] == 0.25
    for r, s in enumerate(sninputs.PIPE_PROBLEMS[2]):
        assert np.all(p.sigma_s[reg == r] == s)
    assert np.allclose(p.sigma_t - p.sigma_s, 1e-3, rtol=0, atol=1e-12)
    q0 = sninputs.crooked_pipe(2, None, cells_per_unit=4)
    assert np.array_equal(q0.sigma_t, q0.sigma_s)            # no absorption
    x = (np.arange(p.ncells) % p.nx + 0.5) * p.h[0]
    assert np.all(reg[p.q > 0] == 0) and np.all(x[p.q > 0] < 1.0) and p.q.sum() > 0
    # the pipe connects the inlet (x = 0) to the outlet (x = 14): flood fill over pipe cells
    pipe = (reg == 0).reshape(p.ny, p.nx)
    seen = np.zeros_like(pipe)
    stack = [(j, 0) for j in range(p.ny) if pipe[j, 0]]
    while stack:
        j, i = stack.pop()
        if seen[j, i]:
            continue
        seen[j, i] = True
        for dj, di in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            jj, ii = j + dj, i + di
            if 0 <= jj < p.ny and 0 <= ii < p.nx and pipe[jj, ii] and not seen[jj, ii]:
                stack.append((jj, ii))
    assert seen[:, -1].any() and seen.sum() == pipe.sum()
