"""Large-n chains (d = 27, n = 729: per-step GEMM launches) and the n just
above each fused kernel's limit, against the FP64 oracle on the same P."""
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


@pytest.fixture(scope="module")
def P27(lb):
    H, Lk = W.transmon_system(3)
    L = lb.liouvillian(T(H), T(Lk))
    return lb.propagator(L, W.DT_NS).cpu().numpy()  # parity of this build is tested elsewhere


def states(d, B, seed):
    g = np.random.default_rng(seed)
    return np.stack([W.wishart_state(d, g) for _ in range(B)]).reshape(B, d * d)


def run(lb, P, X, nsteps, prec):
    x = T(X.copy())
    lb.propagate(T(P), x, nsteps, prec)
    return x.cpu().numpy()


def test_d27_sliced_config3_meets_1e6(lb, P27):
    """Config 3 length (1e3 steps), sliced BF16: trace distance < 1e-6."""
    X = states(27, 8, 11)
    ref = oracle.propagate(P27, X, 1000)
    got = run(lb, P27, X, 1000, "bf16_sliced")
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"sliced d=27 N=1e3: trace distance max {td.max():.3e}")
    assert td.max() < 1e-6


@pytest.mark.parametrize("B", [1, 20, 33])
@pytest.mark.parametrize("prec,tol", [("c64", 5e-5), ("bf16_hilo", 5e-3), ("bf16_sliced", 1e-6), ("c128", 1e-12)])
def test_d27_paths(lb, P27, B, prec, tol):
    X = states(27, B, 100 + B)
    ref = oracle.propagate(P27, X, 60)
    got = run(lb, P27, X, 60, prec)
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"{prec} d=27 B={B} N=60: trace distance max {td.max():.3e}")
    assert td.max() < tol


@pytest.mark.parametrize("n,prec,tol", [(100, "bf16_sliced", 1e-8), (130, "c64", 5e-5), (100, "bf16_hilo", 5e-3),
                                        (90, "c128", 1e-13)])
def test_past_fused_limits(lb, n, prec, tol):
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    P = A / (1.02 * np.linalg.norm(A, 2))
    for B in (3, 37):
        X = g.standard_normal((B, n)) + 1j * g.standard_normal((B, n))
        ref = oracle.propagate(P, X, 30)
        got = run(lb, P, X, 30, prec)
        assert oracle.rel_per_state(got, ref, X) < tol, (B, oracle.rel_per_state(got, ref, X))


def test_d27_deterministic(lb, P27):
    X = states(27, 17, 5)
    for prec in ("c64", "bf16_sliced"):
        a = run(lb, P27, X, 10, prec)
        b = run(lb, P27, X, 10, prec)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,nsteps,tol,variant", [("c128", 200, 1e-12, 1101), ("c64", 200, 5e-5, 1101),
                                                     ("bf16_sliced", 1000, 1e-6, 1202)])
def test_d27_config3_full_batch_sampled(lb, P27, prec, nsteps, tol, variant):
    """Config 3 at its full batch (B = 1024) in the launch configuration the
    bench times (the LDS-tiled step kernels, 256 workgroups); the oracle
    recomputes a sample of states (states are independent)."""
    c = W.config3()
    X = c["rho0"].reshape(1024, 729)
    assert lb.chain_variant(729, prec, 1024) == variant
    got = run(lb, P27, X, nsteps, prec)
    idx = [0, 1, 513, 1023]
    ref = oracle.propagate(P27, X[idx], nsteps)
    g = got[idx]
    if prec == "c128":
        assert oracle.rel_per_state(g, ref) < tol
    td = oracle.trace_distance(g.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"{prec} d=27 B=1024 N={nsteps}: trace distance max {td.max():.3e}")
    assert td.max() < (tol if prec != "c128" else 1e-12)


@pytest.mark.parametrize("prec,nsteps", [("bf16_sliced", 3), ("bf16_sliced", 601), ("bf16_hilo", 3)])
@pytest.mark.parametrize("B", [1024, 100])
def test_ring_plane_kernel_matches_tiled(lb, P27, prec, nsteps, B):
    """The ring-pipelined plane GEMM (1201) does the tiled kernel's (1200)
    arithmetic in the same order with other data movement: results are
    bitwise equal, on the full batch and on a ragged one (B = 100: a partial
    state tile), over a few steps and over several hundred."""
    X = states(27, B, 11 + B)
    out = {}
    for v in (1200, 1201):
        x = T(X.copy())
        lb.propagate_variant(T(P27), x, nsteps, v, prec)
        out[v] = x.cpu().numpy()
    assert np.array_equal(out[1200], out[1201])


@pytest.mark.parametrize("prec", ["bf16_sliced", "bf16_hilo"])
@pytest.mark.parametrize("B,nsteps", [(1024, 3), (100, 3), (64, 601), (1, 20)])
def test_splitk_plane_kernel_matches_ring(lb, P27, prec, B, nsteps):
    """The ring kernel with the k range split over workgroups (1202) against
    the unsplit one (1201): bitwise at 256 tiles (B = 1024: no split).  Else
    the FP64 partial sums of the k ranges are added in order; the state then
    differs by FP64 rounding, which can move the last digit of the next
    step's slicing (2^-32 of the state for the 4-digit state slices) or the
    FP32 rounding of the hi+lo state (2^-24), so the bound is that."""
    X = states(27, B, 21 + B)
    out = {}
    for v in (1201, 1202):
        x = T(X.copy())
        lb.propagate_variant(T(P27), x, nsteps, v, prec)
        out[v] = x.cpu().numpy()
    if B == 1024:
        assert np.array_equal(out[1201], out[1202])
    else:
        scale = np.abs(out[1201]).max()
        tol = 1e-8 if prec == "bf16_sliced" else 1e-5
        assert np.abs(out[1201] - out[1202]).max() <= tol * scale
