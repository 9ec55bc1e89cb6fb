"""The oracle's decisions on the 1000 samples of the small workload (L = 3,
depolarizing p = 0.10, 4 classes x 1 chain) against exact enumeration of every
class (Sec. IV.A: both the single-temperature rule and the 21-temperature
thermodynamic integration approximate the maximum-likelihood class).

Near ties are excluded by a stated band: the chains' own error, measured
against the exact values over all samples (the root mean square of the
estimate minus the exact value, over the two classes the decision is
between), times 5.  Outside that band every decision must equal the exact one,
so the decoder's logical error equals the exact decoder's up to the near-tie
samples.
"""

import numpy as np
import pytest

from oracle import decoder, geometry, sampler, tables
from oracle import enumerate as en

L, P, N = 3, 0.10, 1000
SEED_SMALL = 0x1302266900000001


@pytest.fixture(scope="module")
def workload():
    lat = geometry.Lattice(L)
    syn, cls, _ = sampler.sample(lat, P, SEED_SMALL, np.arange(N))
    bb = tables.beta_bar(P)
    cache = {}
    mean = np.zeros((N, 4))
    prob = np.zeros((N, 4))
    for i in range(N):
        key = syn[i].tobytes()
        if key not in cache:
            h = en.class_histograms(lat, syn[i])
            cache[key] = (en.mean_n(h, bb), en.class_probabilities(h, bb))
        mean[i], prob[i] = cache[key]
    return syn, cls, mean, prob


def test_single_temperature_decisions_match_exact_means(workload):
    """K = 1, 2000 sweeps: the decision is the class with the smallest chain
    average of n (Sec. IV.A), whose exact limit is the argmin of the exact
    <n>_{beta_bar,E}."""
    syn, cls, mean, _ = workload
    out = decoder.decode(L, syn, P, 2000, SEED_SMALL, chains_per_class=1)
    rows = np.arange(N)[:, None]
    top2 = np.argsort(mean, axis=1, kind="stable")[:, :2]
    err = (out["mean_n"] - mean)[rows, top2]
    sigma = float(np.sqrt((err ** 2).mean()))
    band = 5.0 * np.sqrt(2.0) * sigma
    gap = mean[np.arange(N), top2[:, 1]] - mean[np.arange(N), top2[:, 0]]
    exact = top2[:, 0]
    clear = gap >= band
    assert sigma < 0.03, sigma
    assert clear.mean() > 0.85, clear.mean()
    assert np.array_equal(out["chosen"][clear], exact[clear])
    # logical error equal to the exact rule's outside the band
    assert ((out["chosen"] != cls) & clear).sum() == ((exact != cls) & clear).sum()


def test_ti_decisions_match_exact_ml_class(workload):
    """K = 20 (the paper's 21 equidistant temperatures with Simpson's rule),
    200 counted sweeps after 50 of burn-in per temperature: the decision is the
    exact maximum-likelihood class outside the near-tie band."""
    syn, cls, _, prob = workload
    out = decoder.decode(L, syn, P, 200, SEED_SMALL, chains_per_class=1, n_temps=20, burn=50)
    rows = np.arange(N)
    order = np.argsort(-prob, axis=1, kind="stable")
    ml, second = order[:, 0], order[:, 1]
    lx = np.log(prob)
    le = np.log(np.maximum(out["class_prob"], 1e-300))
    est = le[rows, ml] - le[rows, second]
    ex = lx[rows, ml] - lx[rows, second]
    sigma = float(np.sqrt(((est - ex) ** 2).mean()))
    band = 5.0 * sigma
    clear = ex >= band
    assert sigma < 0.15, sigma
    assert clear.mean() > 0.80, clear.mean()
    assert np.array_equal(out["chosen"][clear], ml[clear])
    assert ((out["chosen"] != cls) & clear).sum() == ((ml != cls) & clear).sum()
