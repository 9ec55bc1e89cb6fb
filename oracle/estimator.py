"""Class probabilities by thermodynamic integration, and the decision.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (main): log Z_E(beta_bar) = -int_0^beta_bar <n>_{beta,E} dbeta + n_stab log 2.
Sec. IV.A: as beta -> 0 every qubit is I, X, Y, Z with probability 1/4, so
<n>_{0,E} = (3/4) n_q exactly; that endpoint is used in closed form.

* pooled <n>_{E,k} = (sum over chains of S) / (chains * 4 * sweeps); with no
  counted sweep it is the mean current weight of the chains.  The random
  scan samples n after every one of its n_stab steps per sweep, so there the
  denominator is chains * n_stab * sweeps.
* K = 1 (single temperature, beta* = beta_bar): trapezoid on {0, beta_bar},
  I_E = (beta_bar / 2) (f0 + <n>_{E,1}).
* K = 1 with beta* below beta_bar (the bit/phase-flip model's beta* =
  0.85 beta_bar): the paper does not say how to integrate past the one
  sampled temperature; here the trapezoid covers [0, beta*] and <n> is held
  at its beta* value on [beta*, beta_bar]:
  I_E = (beta* / 2)(f0 + <n>_{E,1}) + (beta_bar - beta*) <n>_{E,1},
  which is the plain trapezoid when beta* = beta_bar.
* Independent bit/phase flips: n is the number of x parts plus z parts, and
  at beta -> 0 each of the 2 n_q parts is set with probability 1/2, so
  f0 = n_q.
* K even (the paper's equidistant temperatures with Simpson's rule):
  h = beta_bar / K, I_E = (h / 3)(f0 + 4 f1 + 2 f2 + ... + 4 f_{K-1} + f_K),
  accumulated in ascending k.
* log Z_E = n_stab log 2 - I_E;  P_E = exp(log Z_E - max) / sum_E' exp(...).
* Decision: the class with the largest Z_E.  Every I_E shares f0 and the
  denominator chains * 4 * sweeps, so this is the class with the smallest
  integer key_E = sum_{k<K} w_k S_{E,k} + S_{E,K} (w_k = 4 for odd k, 2 for
  even k; for K = 1 just S_{E,1}), which for K = 1 is the single-temperature
  rule of Sec. IV.A (smallest <n>_{beta*,E}).  Ties go to the lowest class.
"""

import math

import numpy as np


def simpson_weights(K):
    if K == 1:
        return [1]
    return [4 if k % 2 == 1 else 2 for k in range(1, K)] + [1]


def estimate(S, n_final, chains, sweeps, beta_bar, n_q, n_stab, noise=0, beta_star=None,
             samples_per_sweep=4):
    return estimate_log_z(S, n_final, chains, sweeps, beta_bar, n_q, n_stab, noise,
                          beta_star, samples_per_sweep)[:4]


def estimate_log_z(S, n_final, chains, sweeps, beta_bar, n_q, n_stab, noise=0, beta_star=None,
                   samples_per_sweep=4):
    """S, n_final: int64 [4, K, chains] for one syndrome.

    Returns (class_prob [4], mean_n [4] at the last temperature (beta_bar, or
    beta* for K = 1), key [4] int, chosen int);
    `estimate_log_z` returns the four log Z_E as well.
    """
    S = np.asarray(S, dtype=np.int64)
    n_final = np.asarray(n_final, dtype=np.int64)
    K = S.shape[1]
    T = samples_per_sweep * sweeps
    src = S if T > 0 else n_final
    sums = src.sum(axis=2)                                     # [4, K] exact int
    denom = float(chains * T) if T > 0 else float(chains)
    mean = [[float(sums[e, k]) / denom for k in range(K)] for e in range(4)]
    f0 = float(n_q) if noise == 1 else 0.75 * n_q
    bs = beta_bar if beta_star is None else beta_star
    logz = []
    for e in range(4):
        if K == 1:
            integral = (bs / 2.0) * (f0 + mean[e][0]) + (beta_bar - bs) * mean[e][0]
        else:
            h = beta_bar / K
            acc = f0
            for k in range(1, K):
                acc = acc + (4.0 if k % 2 == 1 else 2.0) * mean[e][k - 1]
            acc = acc + mean[e][K - 1]
            integral = (acc * h) / 3.0
        logz.append(n_stab * math.log(2.0) - integral)
    m = max(logz)
    ex = [math.exp(v - m) for v in logz]
    tot = ((ex[0] + ex[1]) + ex[2]) + ex[3]
    prob = np.array([v / tot for v in ex], dtype=np.float64)
    w = simpson_weights(K)
    key = [sum(int(w[k]) * int(sums[e, k]) for k in range(K)) for e in range(4)]
    chosen = min(range(4), key=lambda e: (key[e], e))
    mean_at_bar = np.array([mean[e][K - 1] for e in range(4)], dtype=np.float64)
    return prob, mean_at_bar, np.array(key, dtype=np.int64), chosen, np.array(logz)
