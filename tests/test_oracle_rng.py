"""Pins of the oracle's counter-based generator and PST template (Sec. 3.3,
Sec. 4 "PST pre-sampling": particles uniform in the unit 6-ball)."""
import math

import numpy as np
import pytest
from scipy import stats


def _np_philox_block(key, ctr):
    """numpy's Philox4x64-10 increments its 256-bit counter before producing
    a block, so the block for counter c is obtained by seeding with c - 1."""
    c = int(ctr[0]) + (int(ctr[1]) << 64) + (int(ctr[2]) << 128) + (int(ctr[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.asarray(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((5600, 0), (1, 0, 0, 0)),
    ((0xDEADBEEF, 123), (7, 9, 11, 13)),
    ((2**64 - 1, 2**63), (2**64 - 1, 2**64 - 1, 5, 0)),
    ((12345, 0), (10239, 1023, 0, 0)),
])
def test_philox_matches_numpy(orc, key, ctr):
    ref = _np_philox_block(key, ctr)
    got = orc.philox4x64_10(ctr, key)
    assert np.array_equal(ref, got)


def test_pst_row0_and_lattice(orc):
    p, capped = orc.pst_sample(4096, 5600)
    assert capped == 0
    assert np.all(p[0] == 0)
    a = p.astype(np.float64) * 2.0**24
    assert np.all(a[1:] == np.round(a[1:]))
    assert np.all(np.abs(a[1:]) % 2 == 1)  # odd lattice points
    s = (a[1:].astype(np.int64) ** 2).sum(1)
    assert np.all(s <= 2**48)


def test_pst_radial_law_and_moments(orc):
    n = 20001
    p, _ = orc.pst_sample(n, 5600)
    x = p[1:].astype(np.float64)
    r6 = np.linalg.norm(x, axis=1) ** 6  # uniform in the 6-ball <=> |p|^6 ~ U(0,1)
    assert stats.kstest(r6, "uniform").pvalue > 1e-3
    m = x.mean(0)
    assert np.all(np.abs(m) < 4 * math.sqrt(1 / 8 / len(x)))
    C = x.T @ x / len(x)  # E[p p^T] = I/8 for the uniform 6-ball
    assert np.allclose(np.diag(C), 1 / 8, atol=0.01)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 0.01
    # per-axis sign symmetry
    frac_pos = (x > 0).mean(0)
    assert np.all(np.abs(frac_pos - 0.5) < 0.02)


def test_pst_seed_changes_template(orc):
    a, _ = orc.pst_sample(64, 1)
    b, _ = orc.pst_sample(64, 2)
    assert not np.array_equal(a[1:], b[1:])
    c, _ = orc.pst_sample(64, 1)
    assert np.array_equal(a, c)


def test_pst_acceptance_rate_and_reconstruction(orc):
    """Rebuild the first rows from numpy's Philox blocks: the accepted
    attempt equals the oracle's row, and the acceptance rate matches the
    6-ball / cube volume ratio pi^3/384."""
    n = 600
    seed = 5600
    p, _ = orc.pst_sample(n, seed)
    tries = 0
    for i in range(1, n):
        for a in range(1024):
            tries += 1
            w = _np_philox_block((seed, 0), (i, a, 0, 0))
            m = [int(w[0]) >> 40, (int(w[0]) >> 16) & 0xFFFFFF, int(w[1]) >> 40, (int(w[1]) >> 16) & 0xFFFFFF,
                 int(w[2]) >> 40, (int(w[2]) >> 16) & 0xFFFFFF]
            av = [2 * v + 1 - 2**24 for v in m]
            if sum(v * v for v in av) <= 2**48:
                assert np.array_equal(p[i], np.array([v * 2.0**-24 for v in av], dtype=np.float32))
                break
    rate = (n - 1) / tries
    expect = math.pi**3 / 384
    sd = math.sqrt(expect * (1 - expect) / tries)
    assert abs(rate - expect) < 4 * sd + 0.005
