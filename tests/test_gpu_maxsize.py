"""The largest supported size, d = 64 (n = 4096): the superoperator against
the oracle element by element, and the propagator and chain through
properties that hold at any size (the oracle's own n = 4096 build would take
hours): trace preservation, Hermiticity preservation, the semigroup law
exp(2A) = exp(A)^2, and the chain against the oracle's matvecs on the same P."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
D = 64
N = D * D


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def lb():
    from paper_2603_18052_amd import lindblad
    lindblad.lib()
    return lindblad


@pytest.fixture(scope="module")
def system():
    g = np.random.default_rng(6464)
    A = g.standard_normal((D, D)) + 1j * g.standard_normal((D, D))
    H = 0.02 * (A + A.conj().T)
    Lk = 0.02 * (g.standard_normal((2, D, D)) + 1j * g.standard_normal((2, D, D)))
    return H, Lk


def test_liouvillian_d64_matches_oracle(lb, system):
    H, Lk = system
    ref = oracle.liouvillian(H, Lk)
    got = lb.liouvillian(T(H), T(Lk)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_propagator_d64_properties_and_chain(lb, system):
    H, Lk = system
    L = lb.liouvillian(T(H), T(Lk))
    dt = 0.5
    P, s = lb.propagator(L, dt, return_s=True)
    P2, s2 = lb.propagator(L, 2 * dt, return_s=True)
    assert s2 == s + 1 or s2 == s  # ||2A|| = 2 ||A||
    # trace preservation: vec(I)^T P = vec(I)^T (row-major vec(I) has ones at i d + i)
    diag = torch.arange(D, device=DEV) * (D + 1)
    tr_rows = P[diag, :].sum(dim=0)
    vecI = torch.zeros(N, dtype=torch.complex128, device=DEV)
    vecI[diag] = 1.0
    assert (tr_rows - vecI).abs().max().item() < 1e-12
    # semigroup: exp(2A) = exp(A)^2 (each side a separate Alg. 1 build)
    PP = P @ P
    rel = ((PP - P2).abs().max() / P2.abs().max()).item()
    assert rel < 1e-12, rel
    # Hermiticity preservation and the chain against the oracle's matvecs
    g = np.random.default_rng(7)
    G = g.standard_normal((3, D, D)) + 1j * g.standard_normal((3, D, D))
    rho = G @ G.conj().transpose(0, 2, 1)
    rho /= np.trace(rho, axis1=1, axis2=2)[:, None, None]
    X = rho.reshape(3, N)
    ref = oracle.propagate(P.cpu().numpy(), X, 3)
    for prec, tol in (("c128", 1e-12), ("c64", 1e-4)):
        x = T(X.copy())
        lb.propagate(P, x, 3, prec)
        got = x.cpu().numpy()
        if prec == "c128":
            assert oracle.rel_per_state(got, ref) < tol
        else:
            assert oracle.trace_distance(got.reshape(3, D, D), ref.reshape(3, D, D)).max() < tol
        m = got.reshape(3, D, D)
        assert np.abs(m - m.conj().transpose(0, 2, 1)).max() < (1e-13 if prec == "c128" else 1e-6)
