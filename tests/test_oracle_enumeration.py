"""Exact pin of the oracle's likelihood increment and resampler: a bootstrap
filter on a two-state hidden Markov model, enumerated outcome by outcome.

The filter's likelihood estimate (Alg. 2: the product over time of the mean
weight, each factor exp(ell_t) with ell_t = M + ln S - ln N) is unbiased for
the marginal likelihood p(y_1, ..., y_T).  With N <= 4 particles and T <= 2
observations every random outcome can be listed: the initial states (2^N
draws), the systematic resampling uniform (the outcome is constant on the
intervals of u between the breakpoints frac(N W_j / S), weighted by their
lengths) and the transitions (2^N draws).  The expectation of
exp(ell_1 + ... + ell_T) over all of them must equal the forward algorithm's
p(y_1:T) to rounding; the oracle's collective (orc_reduce_resample) supplies
every ell_t and every set of ancestors.  A dropped -ln N, a biased set of
ancestors or an increment taken after instead of before resampling all move
the expectation by far more than rounding, and the test checks that the
planted forms do."""
import itertools
import math

import numpy as np
import pytest

import oracle

P0 = np.array([0.3, 0.7])                 # initial law
PT = np.array([[0.9, 0.1], [0.2, 0.8]])   # transition matrix, rows: from
MU = np.array([0.0, 2.0])                 # observation mean per state, sd 1
Y = [0.5, 1.7]


def logg(x, y):
    return -0.5 * (y - MU[x]) ** 2 - 0.5 * math.log(2 * math.pi)


def forward(T):
    """p(y_1:T) by the forward algorithm (the exact answer)."""
    alpha = P0 * np.exp([logg(0, Y[0]), logg(1, Y[0])])
    for t in range(1, T):
        alpha = (alpha @ PT) * np.exp([logg(0, Y[t]), logg(1, Y[t])])
    return float(alpha.sum())


def u_intervals(lw):
    """The intervals of u in [0, 1) on which the systematic ancestors are
    constant, as (midpoint, length) pairs."""
    N = lw.size
    w = np.exp(lw - lw.max())
    cuts = np.unique(np.concatenate([[0.0, 1.0], np.mod(np.cumsum(w) / w.sum() * N, 1.0)]))
    return [(0.5 * (lo + hi), hi - lo) for lo, hi in zip(cuts[:-1], cuts[1:]) if hi - lo > 0]


def expectation(N, T, mistake=None):
    """E[exp(sum_t ell_t)] over every outcome of the bootstrap filter."""
    total = 0.0
    for x1 in itertools.product((0, 1), repeat=N):
        p1 = float(np.prod(P0[list(x1)]))
        total += p1 * branch(np.array(x1), 0, T, N, mistake)
    return total


def branch(x, t, T, N, mistake):
    """Expected exp(sum of the remaining increments) given the particles x
    propagated to time t (0-based), weighted by y_t."""
    lw = np.array([logg(int(s), Y[t]) for s in x])
    st, ell, _, _ = oracle.reduce_resample(lw, 0.5)
    assert st == 0
    if mistake == "no_minus_ln_N":
        ell += math.log(N)
    if t == T - 1:
        return math.exp(ell)
    out = 0.0
    for u, length in u_intervals(lw):
        _, _, _, a = oracle.reduce_resample(lw, u)
        if mistake == "argmax_ancestors":
            a = np.full(N, int(np.argmax(lw)))
        ell_u = ell
        if mistake == "ell_after_resampling":  # the mean weight of the resampled set
            ell_u = oracle.reduce_resample(lw[a], 0.5)[1]
        xa = x[a]
        for x2 in itertools.product((0, 1), repeat=N):
            p2 = float(np.prod(PT[xa, list(x2)]))
            if p2 == 0.0:
                continue
            out += length * p2 * math.exp(ell_u) * branch(np.array(x2), t + 1, T, N, mistake)
    return out


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("T", [1, 2])
def test_likelihood_estimate_is_exactly_unbiased(orc, N, T):
    exact = forward(T)
    got = expectation(N, T)
    assert abs(got - exact) <= 1e-12 * exact, (N, T, got, exact)


@pytest.mark.parametrize("mistake", ["no_minus_ln_N", "argmax_ancestors", "ell_after_resampling"])
def test_planted_mistakes_move_the_expectation(orc, mistake):
    exact = forward(2)
    got = expectation(3, 2, mistake)
    assert abs(got - exact) > 1e-3 * exact, (mistake, got, exact)
