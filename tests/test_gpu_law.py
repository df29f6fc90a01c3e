"""Second check of the GPU engines: their distributions against the exact
master equation, and against each other.

The bit-exact parity tests compare the GPU with the oracle draw for draw.
Here the GPU results are compared with laws that no implementation supplies:
the exact distribution of the uniformised chain (fixed number of events,
dyadic rationals) and of the master equation at time t (Poisson mixture), for
N_tot = 10, with 2^16 replicas per engine: Pearson chi-square on the states
and a one-sample Kolmogorov-Smirnov test on the enantiomeric excess (exact
for continuous laws, conservative for this discrete one).  The plain engine
draws its own random numbers (PLAIN domain), so a two-sample test between it
and the bit-sliced engine compares two independent samples of one law.
"""

import numpy as np
import pytest
from scipy import stats

import paper_2412_16613_amd as bwg
from oracle import master
from oracle.quantize import quantize
from workloads import frank_network, paper_network

pytestmark = pytest.mark.gpu

M = 1 << 16
P_MIN = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def chi2_pvalue(observed, expected, min_expected=5.0):
    """Pearson chi-square with cells of small expectation pooled."""
    observed = np.asarray(observed, float)
    expected = np.asarray(expected, float)
    obs_p, exp_p = [], []
    acc_o = acc_e = 0.0
    for i in np.argsort(expected):
        acc_o += observed[i]
        acc_e += expected[i]
        if acc_e >= min_expected:
            obs_p.append(acc_o)
            exp_p.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and exp_p:
        obs_p[-1] += acc_o
        exp_p[-1] += acc_e
    obs_p, exp_p = np.array(obs_p), np.array(exp_p)
    return stats.chi2.sf(((obs_p - exp_p) ** 2 / exp_p).sum(), max(1, len(obs_p) - 1))


def ks_ee_pvalue(counts, st, probs, n_tot):
    """One-sample KS of ee = (N_L - N_D) / N_tot against the law of the states
    st with probabilities probs (the supremum is taken at the support points,
    where the step CDFs jump)."""
    d_law = np.array([s[0] - s[1] for s in st])
    support = np.arange(-n_tot, n_tot + 1)
    F = np.array([probs[d_law <= x].sum() for x in support])
    d = counts[:, 0].astype(np.int64) - counts[:, 1].astype(np.int64)
    Fe = np.searchsorted(np.sort(d), support, side="right") / len(d)
    D = np.max(np.abs(Fe - F))
    return stats.kstwo.sf(D, len(d))


def empirical(counts, st):
    idx = {s: i for i, s in enumerate(st)}
    obs = np.zeros(len(st))
    keys, n = np.unique(counts, axis=0, return_counts=True)
    for k, c in zip(keys, n):
        obs[idx[tuple(int(x) for x in k)]] += c
    return obs


def run(torch, net, engine, init, sched, seed):
    print("law case", engine, net["n_tot"], init, sched, seed, flush=True)
    e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=77, engine=engine)
    e.init(init)
    for op, v in sched:
        getattr(e, op)(v)
    c = e.read_counts().cpu().numpy()
    torch.cuda.synchronize()
    assert (c.sum(1) == net["n_tot"]).all()
    return c


CASES = [
    # Frank network with conversions, fixed number of uniformised events
    ("fixed-K", frank_network(10, k0=0.05), (0, 0, 10), [("step", 150), ("step", 151)]),
    # the same network at time t over two advances (Poisson mixture of the chain)
    ("time", frank_network(10, k0=0.05), (0, 0, 10), [("advance", 4.0), ("advance", 9.0)]),
    # the paper's network with its ghosts (Eq. (9)), unit weights
    ("fixed-K", paper_network(10), (3, 3, 4), [("step", 37)]),
]


def law(net, mode, start, sched):
    q = quantize(net)
    if mode == "fixed-K":
        K = sum(v for _, v in sched)
        return master.fixed_k_probs(net, q, start, K)
    return master.time_probs(net, q, {start: 1.0}, sched[-1][1])


@pytest.mark.parametrize("engine", ["bitwise", "lanes", "plain"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_engine_samples_the_master_equation(torch, engine, case):
    mode, net, start, sched = CASES[case]
    counts = run(torch, net, engine, ("fixed", start), sched, seed=31 + case)
    st, probs = law(net, mode, start, sched)
    assert abs(probs.sum() - 1) < 1e-9
    p_chi2 = chi2_pvalue(empirical(counts, st), probs * M)
    p_ks = ks_ee_pvalue(counts, st, probs, net["n_tot"])
    print("chi2 p = %.3g, KS p = %.3g" % (p_chi2, p_ks), flush=True)
    assert p_chi2 > P_MIN and p_ks > P_MIN


@pytest.mark.parametrize("case", range(len(CASES)))
def test_bitwise_and_plain_engines_agree(torch, case):
    # independent draws (EVENT planes against PLAIN words): a two-sample
    # chi-square on the states and a two-sample KS on ee
    mode, net, start, sched = CASES[case]
    a = run(torch, net, "bitwise", ("fixed", start), sched, seed=51 + case)
    b = run(torch, net, "plain", ("fixed", start), sched, seed=51 + case)
    st, probs = law(net, mode, start, sched)
    oa, ob = empirical(a, st), empirical(b, st)
    # states pooled in order of probability until each pool expects >= 5
    # replicas per sample
    pools, cur, acc = [], [], 0.0
    for i in np.argsort(probs):
        cur.append(i)
        acc += probs[i] * M
        if acc >= 5.0:
            pools.append(cur)
            cur, acc = [], 0.0
    if cur:
        pools[-1] += cur
    table = np.array([[oa[p].sum() for p in pools], [ob[p].sum() for p in pools]])
    p_chi2 = stats.chi2_contingency(table)[1]
    ea = (a[:, 0] - a[:, 1]).astype(np.int64)
    eb = (b[:, 0] - b[:, 1]).astype(np.int64)
    p_ks = stats.ks_2samp(ea, eb).pvalue
    print("two-sample chi2 p = %.3g, KS p = %.3g" % (p_chi2, p_ks), flush=True)
    assert p_chi2 > P_MIN and p_ks > P_MIN
