"""GPU parity of the Hermitian-coordinate INT8-digit chain (LB_I8_HERM)
against the CPU oracle.

The Lindblad generator of Eq. (1) maps rho^dagger to (L rho)^dagger, and so
does every propagator built from it by the Pade-13 scaling and squaring of
Alg. 1 (real coefficients), so a density matrix stays Hermitian along the
chain of Alg. 2.  LB_I8_HERM runs the step on the d^2 real coordinates of the
state (Re rho_ij on and above the diagonal, Im rho_ij below it) with the
same digits and rules as LB_I8_SLICED.  The oracle knows nothing of that
form: it runs the plain complex chain, and the tests compare the states.
"""
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
    assert torch.cuda.is_available()
    return lindblad


@pytest.fixture(scope="module")
def P9():
    H, Lk = W.transmon_system(2)
    return oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)


@pytest.fixture(scope="module")
def P3():
    H, Lk = W.transmon_system(1)
    return oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)


def states(d, B, seed):
    g = np.random.default_rng(seed)
    return np.stack([W.wishart_state(d, g) for _ in range(B)]).reshape(B, d * d)


def kraus_map(d, g, k=3, gain=0.98):
    """A random Hermiticity-preserving map on row-major vec: sum_k A_k (x) conj(A_k)
    (vec(A rho A^dagger)), scaled to spectral norm `gain`."""
    P = np.zeros((d * d, d * d), complex)
    for _ in range(k):
        A = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
        P += np.kron(A, A.conj())
    return P * (gain / np.linalg.norm(P, 2))


def hermitian_states(d, B, g):
    X = g.standard_normal((B, d, d)) + 1j * g.standard_normal((B, d, d))
    return (0.5 * (X + X.conj().transpose(0, 2, 1))).reshape(B, d * d)


def run(lb, P, X, nsteps, variant=None):
    x = T(X.copy())
    if variant is None:
        lb.propagate(T(P), x, nsteps, "i8_herm")
    else:
        lb.propagate_variant(T(P), x, nsteps, variant, "i8_herm")
    return x.cpu().numpy()


def assert_hermitian(X, d):
    R = X.reshape(-1, d, d)
    assert np.array_equal(R, R.conj().transpose(0, 2, 1))


def test_herm_single_step(lb, P9):
    """One step against P x: the error of 30-bit coordinates and 38-bit
    row-scaled digits of the real step matrix."""
    X = states(9, 16, 3)
    got = run(lb, P9, X, 1)
    err = np.abs(got - X @ P9.T).max()
    print(f"i8 herm one step: max abs error {err:.3e}")
    assert err < 2e-9
    assert_hermitian(got, 9)


@pytest.mark.parametrize("nsteps", [1000, 10000])
def test_herm_d9_meets_1e6(lb, P9, nsteps):
    X = states(9, 37, 41)  # two full workgroups and a ragged one
    ref = oracle.propagate(P9, X, nsteps)
    got = run(lb, P9, X, nsteps)
    td = oracle.trace_distance(got.reshape(-1, 9, 9), ref.reshape(-1, 9, 9))
    print(f"i8 herm d=9 N={nsteps}: trace distance max {td.max():.3e} median {np.median(td):.3e}")
    assert td.max() < 1e-6
    assert_hermitian(got, 9)
    rep = oracle.state_report(got.reshape(-1, 9, 9))
    assert rep["trace_err"].max() < 1e-6 and rep["lambda_min"].min() > -1e-6


def test_herm_d3_config1(lb, P3):
    c = W.config1()
    ref = oracle.propagate(P3, c["rho0"].reshape(1, 9), c["nsteps"])
    got = run(lb, P3, c["rho0"].reshape(1, 9), c["nsteps"])
    td = oracle.trace_distance(got.reshape(3, 3), ref.reshape(3, 3))
    print(f"i8 herm d=3 N=1e4: trace distance {td:.3e}")
    assert td < 1e-6


@pytest.mark.parametrize("d", [1, 2, 5, 8, 9, 10, 11, 12, 13])
def test_herm_shapes(lb, d):
    """Every tile count (1 .. 11 row tiles of the n x n real step, 1 .. 3 k
    chunks) on a random Hermiticity-preserving contraction, 19 Hermitian
    (indefinite) states: a ragged workgroup."""
    g = np.random.default_rng(200 + d)
    P = kraus_map(d, g)
    X = hermitian_states(d, 19, g)
    ref = oracle.propagate(P, X, 40)
    got = run(lb, P, X, 40)
    assert oracle.rel_per_state(got, ref, X) < 1e-8
    assert_hermitian(got, d)


@pytest.mark.parametrize("d", [3, 9, 13])
def test_herm_fused_forms_agree_bitwise(lb, d):
    """1300 / 1301 / 1302 give the same bits in the Hermitian form too, also
    under a growing map that makes every step re-slice."""
    g = np.random.default_rng(300 + d)
    n = d * d
    P = kraus_map(d, g)
    X = hermitian_states(d, 37, g)
    for Pm, steps in ((P, 50), (3.0 * np.eye(n, dtype=complex) + 0.01 * P, 20)):
        out = {v: run(lb, Pm, X, steps, v) for v in (1300, 1301, 1302)}
        for v in (1301, 1302):
            assert np.array_equal(out[1300], out[v]), v
        ref = oracle.propagate(Pm, X, steps)
        assert oracle.rel_per_state(out[1302], ref, X) < 1e-8


def test_herm_reads_upper_real_and_lower_imaginary(lb):
    """A non-Hermitian input: the call propagates the Hermitian matrix of its
    coordinates (Re x_ij for i <= j, Im x_ij for i > j), deterministically,
    and a zero state stays zero."""
    d, B = 4, 6
    g = np.random.default_rng(7)
    P = kraus_map(d, g)
    X = (g.standard_normal((B, d, d)) + 1j * g.standard_normal((B, d, d)))
    X[2] = 0.0
    Hm = np.zeros_like(X)
    for i in range(d):
        Hm[:, i, i] = X[:, i, i].real
        for j in range(i + 1, d):
            Hm[:, i, j] = X[:, i, j].real - 1j * X[:, j, i].imag
            Hm[:, j, i] = np.conj(Hm[:, i, j])
    X, Hm = X.reshape(B, -1), Hm.reshape(B, -1)
    got = run(lb, P, X, 30)
    assert np.array_equal(got, run(lb, P, X, 30))
    assert not got[2].any()
    ref = oracle.propagate(P, Hm, 30)
    keep = np.arange(B) != 2
    assert oracle.rel_per_state(got[keep], ref[keep], Hm[keep]) < 1e-8


def test_herm_shape_errors(lb, P9):
    """n must be a perfect square."""
    x = T(np.zeros((2, 82), complex))
    with pytest.raises(lb.LindbladError):
        lb.propagate(T(np.eye(82, dtype=complex)), x, 1, "i8_herm")
    x = T(np.zeros((2, 200), complex))
    with pytest.raises(lb.LindbladError):
        lb.propagate(T(np.eye(200, dtype=complex)), x, 1, "i8_herm")


def test_herm_config2_full_size(lb, P9):
    """The bench's configuration (4096 Wishart states, 1e4 steps): the three
    fused forms give the same bits, and sampled states match the oracle's
    chain on the same P."""
    c = W.config2()
    X = c["rho0"].reshape(-1, 81)
    out = {v: run(lb, P9, X, c["nsteps"], v) for v in (1300, 1301, 1302)}
    assert np.array_equal(out[1300], out[1301]) and np.array_equal(out[1300], out[1302])
    idx = np.array([0, 1, 15, 16, 777, 2048, 4094, 4095])
    ref = oracle.propagate(P9, X[idx], c["nsteps"])
    td = oracle.trace_distance(out[1300][idx].reshape(-1, 9, 9), ref.reshape(-1, 9, 9))
    print(f"i8 herm config 2 (B=4096, N=1e4) sampled: trace distance max {td.max():.3e}")
    assert td.max() < 1e-6
    assert_hermitian(out[1300], 9)


@pytest.mark.parametrize("d", [14, 15, 20])
def test_herm_gemm_shapes_agree_bitwise(lb, d):
    """Past the fused limit (n = d^2 > 192) the per-step INT8 GEMM runs the
    n x n Hermitian step: every tile shape (1500 .. 1503) gives the same
    bits, within the representation's bound of the oracle's chain, and a
    Hermitian result."""
    g = np.random.default_rng(400 + d)
    P = kraus_map(d, g)
    X = hermitian_states(d, 19, g)
    out = {v: run(lb, P, X, 20, v) for v in (1500, 1501, 1502, 1503)}
    for v in (1501, 1502, 1503):
        assert np.array_equal(out[1500], out[v]), v
    ref = oracle.propagate(P, X, 20)
    assert oracle.rel_per_state(out[1500], ref, X) < 1e-8
    assert_hermitian(out[1500], d)


@pytest.fixture(scope="module")
def P27():
    H, Lk = W.transmon_system(3)
    return oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)


def test_herm_gemm_d27_config3(lb, P27):
    """Config 3 (d = 27, 10^3 steps) on the oracle's P, a ragged batch: the
    trace distance against the oracle's chain."""
    X = states(27, 37, 17)
    ref = oracle.propagate(P27, X, 1000)
    got = run(lb, P27, X, 1000)
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"i8 herm GEMM d=27 B=37 N=1e3: trace distance max {td.max():.3e} median {np.median(td):.3e}")
    assert td.max() < 1e-6
    assert_hermitian(got, 27)


@pytest.mark.parametrize("B", [1, 64, 1024])
def test_herm_gemm_d27_full_batch_sampled(lb, P27, B):
    c = W.config3(B=B)
    X = c["rho0"].reshape(-1, 729)
    idx = np.unique(np.array([0, 1, 63, 64, 700, 1023]) % B)
    ref = oracle.propagate(P27, X[idx], c["nsteps"])
    got = run(lb, P27, X, c["nsteps"])[idx]
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"i8 herm GEMM config 3 B={B} sampled: trace distance max {td.max():.3e}")
    assert td.max() < 1e-6
