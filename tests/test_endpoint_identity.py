"""CPU check of the identity the GPU build relies on: the closed-form coefficients of section 2.3.1 equal
same-signed weighted sums of two endpoint masses per fragment (a (1 - t) at endpoint j, a t at j + 1, with
u = M x, j = min(floor(u), M - 1), t = u - j), because 1 - x and every tent are linear on a finest cell.
The reference is the oracle's direct N + 2 update per fragment."""
import numpy as np
import pytest


def endpoint_coeffs(rank, x, a):
    M = 2 ** (rank + 1)
    e = np.zeros(M + 1)
    u = M * np.asarray(x, float)
    j = np.minimum(np.floor(u), M - 1).astype(int)
    t = u - j
    np.add.at(e, j, a * (1 - t))
    np.add.at(e, j + 1, a * t)
    cf = np.zeros(M)
    m = np.arange(M + 1)
    cf[0] = (e * (M - m) / M).sum()
    for n in range(rank + 1):
        s = 2 ** n
        w = M // s
        for k in range(s):
            i = np.arange(w + 1)
            tau = np.where(2 * i <= w, i, w - i) / w
            cf[s + k] = -(e[k * w:(k + 1) * w + 1] * tau).sum()
    return cf, e.sum()


@pytest.mark.parametrize("rank", [0, 1, 2, 3, 4, 5])
def test_endpoint_masses_reproduce_closed_forms(orc, rank):
    rng = np.random.default_rng(rank)
    M = 2 ** (rank + 1)
    for trial in range(25):
        k = int(rng.integers(1, 60))
        x = rng.uniform(0, 1, k)
        if trial == 0:
            x[: min(k, 4)] = [0.0, 1.0, 0.5, min(3 / M, 1.0)][: min(k, 4)]
        a = -np.log1p(-rng.uniform(0.01, 0.9, k))
        direct = orc.coeffs_one(rank, x, a)
        cf, tot = endpoint_coeffs(rank, x, a)
        np.testing.assert_allclose(cf, direct, rtol=1e-12, atol=1e-14)
        assert tot == pytest.approx(a.sum(), rel=1e-13)
