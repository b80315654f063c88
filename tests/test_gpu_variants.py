"""Every chain variant (kernel family x tile shape) the library lists for a
shape, against the oracle's FP64 chain on the same P (the oracle's own build,
so only the chain is compared), plus the autotuner's bookkeeping."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_18052_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"c128": 1e-12, "c64": 1e-4, "bf16_hilo": 5e-3, "bf16_sliced": 1e-6}


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def lb():
    from paper_2603_18052_amd import lindblad
    lindblad.lib()
    return lindblad


_P = {}


def oracle_P(d):
    """The oracle's propagator of the transmon model (d = 3, 9, 27) or of a
    random Lindbladian with one collapse operator (d = 2, 4)."""
    if d not in _P:
        if d in (3, 9, 27):
            H, Lk = W.transmon_system({3: 1, 9: 2, 27: 3}[d])
        else:
            g = np.random.default_rng(40 + d)
            A = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
            H = 0.1 * (A + A.conj().T)
            Lk = (0.05 * (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))))[None]
        _P[d] = oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)
    return _P[d]


def states(d, B, seed):
    g = np.random.default_rng(seed)
    return np.stack([W.wishart_state(d, g) for _ in range(B)]).reshape(B, d * d)


# step counts above 2 x 32 + 1 so that the graph-replayed variants replay
CASES = [(2, 5, 200), (3, 1, 300), (3, 20, 300), (4, 70, 200), (9, 1, 200), (9, 20, 200), (27, 3, 70), (27, 20, 70)]


@pytest.mark.parametrize("prec", ["c128", "c64", "bf16_hilo", "bf16_sliced"])
@pytest.mark.parametrize("d,B,N", CASES)
def test_every_variant_matches_oracle(lb, d, B, N, prec):
    n = d * d
    P = oracle_P(d)
    X = states(d, B, 7 * d + B)
    ref = oracle.propagate(P, X, N)
    variants = lb.chain_variants(n, prec, B)
    assert variants
    Pt = T(P)
    for v in variants:
        x = T(X.copy())
        lb.propagate_variant(Pt, x, N, v, prec)
        got = x.cpu().numpy()
        if prec == "c128":
            err = oracle.rel_per_state(got, ref)
        else:
            err = oracle.trace_distance(got.reshape(-1, d, d), ref.reshape(-1, d, d)).max()
        print(f"d={d} B={B} N={N} {prec} {lb.variant_name(v)}: {err:.2e}")
        assert err < TOL[prec], (lb.variant_name(v), err)


def test_variant_runs_are_deterministic_and_zero_steps(lb):
    P = T(oracle_P(9))
    X = states(9, 20, 3)
    for v in lb.chain_variants(81, "c128", 20):
        a, b = T(X.copy()), T(X.copy())
        lb.propagate_variant(P, a, 50, v, "c128")
        lb.propagate_variant(P, b, 50, v, "c128")
        assert torch.equal(a, b), lb.variant_name(v)
        z = T(X.copy())
        lb.propagate_variant(P, z, 0, v, "c128")
        assert np.array_equal(z.cpu().numpy(), X)


def test_wave_chain_config1_full_length(lb):
    """Config 1 (d = 3, one pure state, 1e4 steps) on the one-wavefront chain."""
    c = W.config1()
    P = oracle_P(3)
    X = c["rho0"].reshape(1, 9)
    ref = oracle.propagate(P, X, c["nsteps"])
    x = T(X.copy())
    lb.propagate_variant(T(P), x, c["nsteps"], 200, "c128")
    got = x.cpu().numpy()
    assert oracle.rel_per_state(got, ref) < 1e-12
    assert oracle.trace_distance(got.reshape(3, 3), ref.reshape(3, 3)) < 1e-12


@pytest.mark.parametrize("d,B,prec", [(3, 1, "c128"), (9, 33, "c128"), (27, 20, "c64")])
def test_tune_records_a_listed_variant(lb, d, B, prec):
    n = d * d
    P = T(oracle_P(d))
    X = states(d, B, 11)
    x = T(X.copy())
    best, ms = lb.tune(P, x, prec, probe_steps=8, repeats=2)
    assert best in lb.chain_variants(n, prec, B) and ms > 0
    assert np.array_equal(x.cpu().numpy(), X)  # the tuner works on a copy
    assert lb.chain_variant(n, prec, B) == best
    ref = oracle.propagate(oracle_P(d), X, 30)
    lb.propagate(P, x, 30, prec)
    got = x.cpu().numpy()
    if prec == "c128":
        assert oracle.rel_per_state(got, ref) < 1e-12
    else:
        assert oracle.trace_distance(got.reshape(-1, d, d), ref.reshape(-1, d, d)).max() < 1e-4
    lb.tune_set(n, prec, B, 0)
    assert lb.chain_variant(n, prec, B) != 0


@pytest.mark.parametrize("d,B,prec", [(9, 20, "c128"), (27, 3, "c64"), (9, 17, "bf16_sliced"), (27, 2, "bf16_hilo")])
@pytest.mark.parametrize("N", [64, 65, 97, 130])
def test_graph_replay_matches_direct_launches(lb, d, B, N, prec):
    """A graph-replayed variant runs exactly the kernels of its direct twin
    (32 captured steps replayed, the rest and the last step direct): the
    results must be bitwise equal, for step counts on both sides of the
    replay boundaries and of both parities."""
    n = d * d
    P = T(oracle_P(d))
    X = states(d, B, 5)
    graph = [v for v in lb.chain_variants(n, prec, B) if v % 100 >= lb.GRAPH_VARIANT and v // 100 in (1, 5, 6, 7, 11, 12)]
    assert graph
    for v in graph:
        a, b = T(X.copy()), T(X.copy())
        lb.propagate_variant(P, a, N, v - lb.GRAPH_VARIANT, prec)
        lb.propagate_variant(P, b, N, v, prec)
        assert torch.equal(a, b), (lb.variant_name(v), N)
