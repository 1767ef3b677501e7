"""6D Poisson-disk PST in the oracle (Sec. 4 "PST pre-sampling"): dart
throwing over the i.i.d. sampler's candidate stream.

Pins (none re-types the oracle's loop):
* r_min = 0 accepts every candidate, so the template is the i.i.d.
  template itself, bit for bit (special case reducing to the tested sampler);
* every pair of output points is at least r_min apart, checked exactly on
  the integer lattice with numpy;
* every candidate drawn and rejected lies within r_min of a point accepted
  before it (the sample is maximal for the candidates it has seen), with the
  candidate stream taken from the i.i.d. sampler;
* a candidate budget too small for n returns fewer rows and zero padding;
* the sample is spread like a uniform one (centred, second moments near
  the uniform ball's 1/8) while its minimum spacing is far above the i.i.d.
  template's.
"""
import numpy as np
import pytest

SCALE = float(2 ** 24)


def lattice(p):
    return np.rint(np.asarray(p, np.float64) * SCALE).astype(np.int64)


def min_pair_d2(a):
    best = None
    for i in range(1, len(a)):
        d = a[:i] - a[i]
        s = int(np.min(np.sum(d * d, axis=1)))
        best = s if best is None else min(best, s)
    return best


def test_zero_radius_is_the_iid_template(orc):
    P, got, drawn = orc.pst_poisson(777, 5600, 0.0, 1000)
    iid, _ = orc.pst_sample(777, 5600)
    assert got == 777 and drawn == 776
    assert np.array_equal(P.view(np.uint32), iid.view(np.uint32))


@pytest.mark.parametrize("n,seed,r", [(300, 3, 0.35), (1024, 5600, 0.3)])
def test_minimum_spacing_and_maximality(orc, n, seed, r):
    P, got, drawn = orc.pst_poisson(n, seed, r, 200000)
    assert got == n and drawn >= n - 1
    a = lattice(P)
    assert np.all(a[0] == 0)
    d2 = int(np.ceil(r * r * 2.0 ** 48))
    assert min_pair_d2(a) >= d2
    # the candidate stream: rows 1..drawn of the i.i.d. sampler
    cand = lattice(orc.pst_sample(drawn + 1, seed)[0])[1:]
    acc_rows = {tuple(x) for x in a}
    acc_list = [a[0]]
    for c in cand:
        if tuple(c) in acc_rows and np.min(np.sum((np.array(acc_list) - c) ** 2, axis=1)) >= d2:
            acc_list.append(c)
            continue
        # rejected: some earlier accepted point is within r
        assert np.min(np.sum((np.array(acc_list) - c) ** 2, axis=1)) < d2
    assert len(acc_list) == n
    assert np.array_equal(np.array(acc_list), a)


def test_budget_exhaustion_pads_with_zeros(orc):
    P, got, drawn = orc.pst_poisson(1000, 9, 0.45, 500)
    assert got < 1000 and drawn == 500
    assert np.all(P[got:] == 0) and np.any(P[got - 1] != 0)


def test_spread_like_uniform(orc):
    P, got, _ = orc.pst_poisson(4096, 77, 0.28, 400000)
    iid, _ = orc.pst_sample(4096, 77)
    assert got == 4096
    p = P.astype(np.float64)
    assert np.all(np.abs(p.mean(0)) < 0.02)
    m2 = (p ** 2).mean(0)
    assert np.all((m2 > 0.115) & (m2 < 0.145))  # uniform ball: 1/8 per axis
    assert np.all(np.linalg.norm(p, axis=1) <= 1.0)
    assert min_pair_d2(lattice(P)) > 4 * min_pair_d2(lattice(iid))
