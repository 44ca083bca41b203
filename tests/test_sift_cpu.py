"""Library sifting (host code, no GPU) against the oracle's reading, exactly."""
import numpy as np
import pytest

import oracle as O


def _random_list(seed, n, nseries=12, T=(52.4288, 26.2144)):
    import paper_1912_12807_amd as F
    rng = np.random.default_rng(seed)
    c = np.zeros(n, F.CAND_DTYPE)
    base = rng.uniform(1.0, 60.0, max(1, n // 12))           # a few "signals"
    for i in range(n):
        s = int(rng.integers(0, nseries))
        Ts = T[s % len(T)]
        kind = rng.random()
        if kind < 0.5:                                        # near a signal (duplicate)
            f = base[rng.integers(0, len(base))] + rng.normal(0, 0.7) / Ts
        elif kind < 0.8:                                      # a harmonic or subharmonic of one
            nh = int(rng.integers(2, 20))
            b = base[rng.integers(0, len(base))]
            f = (b * nh if rng.random() < 0.5 else b / nh) + rng.normal(0, 0.5) / Ts
        else:
            f = rng.uniform(0.5, 200.0)
        f = abs(f) + 0.05
        c[i]["series"], c[i]["harm"] = s, int(2 ** rng.integers(0, 4))
        c[i]["r_idx"] = int(rng.integers(0, 1 << 20))
        c[i]["sigma"] = round(float(rng.uniform(6, 12)), 1)   # ties on purpose
        c[i]["f_hz"] = f
        c[i]["r_fund"] = f * Ts
    return c


@pytest.mark.parametrize("seed,n,tol,mr", [(1, 50, 1.1, 16), (2, 400, 1.1, 16), (3, 400, 2.5, 4), (4, 1500, 0.6, 8),
                                          (5, 1, 1.1, 16), (6, 300, 1.1, 1)])
def test_sift_matches_oracle(seed, n, tol, mr):
    import paper_1912_12807_amd as F
    c = _random_list(seed, n)
    got = F.sift(c, tol, mr)
    ref = O.sift(c, tol, mr)
    assert [tuple(int(v) for v in r) for r in got[["index", "hits", "series_lo", "series_hi"]]] == \
        [(i, h, lo, hi) for i, h, lo, hi in ref]
    assert got["hits"].sum() <= n


def test_sift_empty_and_invalid():
    import paper_1912_12807_amd as F
    assert len(F.sift(np.zeros(0, F.CAND_DTYPE))) == 0
    c = _random_list(7, 5)
    c[2]["f_hz"] = 0.0
    with pytest.raises(F.FdasError):
        F.sift(c)
