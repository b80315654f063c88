"""Action of the exponential (lindblad_expmv): rho <- (e^{tL})^N rho with no
propagator, against the oracle's dense propagator (Pade 13 + LU, pinned in
test_oracle) applied to the same states."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2603_18052_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def lb():
    from paper_2603_18052_amd import lindblad
    lindblad.lib()
    return lindblad


def states(d, B, seed):
    g = np.random.default_rng(seed)
    return np.stack([W.wishart_state(d, g) for _ in range(B)]).reshape(B, d * d)


def shifted_norm(L, t):
    mu = np.trace(L) / L.shape[0]
    return abs(t) * np.abs(L - mu * np.eye(L.shape[0])).sum(axis=0).max()


@pytest.mark.parametrize("q,B,N", [(1, 1, 1), (1, 7, 5), (2, 5, 3), (2, 20, 2), (3, 3, 2), (3, 9, 1)])
def test_expmv_transmon_matches_oracle(lb, q, B, N):
    H, Lk = W.transmon_system(q)
    d = 3 ** q
    L = oracle.liouvillian(H, Lk)
    X = states(d, B, 40 + q)
    ref = oracle.propagate(oracle.propagator(L, W.DT_NS), X, N)
    x = T(X.copy())
    prods = lb.expmv(T(L), x, W.DT_NS, N)
    s, m = lb.expmv_params(shifted_norm(L, W.DT_NS))
    assert prods == s * m
    err = oracle.rel_per_state(x.cpu().numpy(), ref)
    print(f"expmv d={d} B={B} N={N}: {s} x {m} products per step, rel err {err:.2e}")
    assert err < 1e-12


def test_expmv_d27_full_batch_sampled(lb):
    """B = 1024 (the LDS-tiled products); the oracle recomputes sampled states."""
    H, Lk = W.transmon_system(3)
    L = oracle.liouvillian(H, Lk)
    c = W.config3()
    X = c["rho0"].reshape(1024, 729)
    x = T(X.copy())
    lb.expmv(T(L), x, W.DT_NS, 2)
    idx = [0, 100, 1023]
    ref = oracle.propagate(oracle.propagator(L, W.DT_NS), X[idx], 2)
    err = oracle.rel_per_state(x.cpu().numpy()[idx], ref)
    print(f"expmv d=27 B=1024: rel err {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("n,scale", [(50, 40.0), (17, 3.0)])
def test_expmv_nonnormal_generator(lb, n, scale):
    """A non-normal generator with a large norm: many sub-steps."""
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    A = scale * A / np.abs(A).sum(axis=0).max() - 0.3 * scale * np.eye(n)
    X = g.standard_normal((4, n)) + 1j * g.standard_normal((4, n))
    ref = oracle.propagate(oracle.propagator(A, 1.0), X, 1)
    x = T(X.copy())
    lb.expmv(T(A), x, 1.0, 1)
    err = oracle.rel_per_state(x.cpu().numpy(), ref, X)
    print(f"expmv random n={n} ||A||={scale}: rel err {err:.2e}")
    assert err < 1e-12


def test_expmv_degenerate(lb):
    H, Lk = W.transmon_system(1)
    L = oracle.liouvillian(H, Lk)
    X = states(3, 4, 7)
    x = T(X.copy())
    assert lb.expmv(T(L), x, 0.0, 3) >= 1  # t = 0: the identity
    assert np.array_equal(x.cpu().numpy(), X)
    x = T(X.copy())
    lb.expmv(T(L), x, W.DT_NS, 0)  # no steps
    assert np.array_equal(x.cpu().numpy(), X)
    with pytest.raises(lb.LindbladError):
        lb.expmv(T(L), T(X.copy()), float("inf"), 1)
