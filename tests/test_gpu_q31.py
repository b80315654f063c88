"""Fixed-point chain at 31 fraction bits (LB_Q31, Alg. 5 with the paper's
Q1.31 word) on the INT8 matrix cores: bit-exact against the oracle's
128-bit integer chain (integer sums do not depend on their order), on the
paper's d = 3 drift model over its step counts, on transmon propagators,
with saturation forced, and within the paper's Q1.31 drift bound (trace
distance below 1e-5 over 1e4 steps, the fixed-point drift figure)."""
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


def codes(x):
    """Q1.31 codes of the GPU result (its values are integers / 2^31 exactly)."""
    x = x.cpu().numpy()
    re, im = np.rint(np.ldexp(x.real, 31)), np.rint(np.ldexp(x.imag, 31))
    assert np.array_equal(np.ldexp(re, -31), x.real) and np.array_equal(np.ldexp(im, -31), x.imag)
    return re.astype(np.int64), im.astype(np.int64)


def check(lb, P, X, N):
    ref_r, ref_i = oracle.propagate_q31(P, X, N)
    x = T(X.copy())
    lb.propagate(T(P), x, N, "q31")
    r, i = codes(x)
    assert np.array_equal(r, ref_r.reshape(r.shape)) and np.array_equal(i, ref_i.reshape(i.shape)), N
    return x.cpu().numpy()


@pytest.mark.parametrize("drive", [0.0, 0.05])
@pytest.mark.parametrize("N", [1, 10, 100, 1000, 10000])
def test_q31_paper_drift_model(lb, drive, N):
    H, Lk, dt, rho0 = W.paper_fixed_point_model(drive)
    P = oracle.propagator(oracle.liouvillian(H, Lk), dt)
    got = check(lb, P, rho0.reshape(1, 9), N)
    ref = oracle.propagate(P, rho0.reshape(1, 9), N)
    td = oracle.trace_distance(got.reshape(3, 3), ref.reshape(3, 3))
    loss = abs(np.trace(got.reshape(3, 3)).real - 1.0)
    assert td < 1e-5 and loss < 1e-5  # the paper's Q1.31 curve stays below 1e-5 over 1e4 steps


@pytest.mark.parametrize("q,B,N", [(1, 37, 500), (2, 20, 200)])
def test_q31_transmon_chains(lb, q, B, N):
    d = 3 ** q
    H, Lk = W.transmon_system(q)
    P = oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)
    X = W.wishart_batch(d, B, 70 + q).reshape(B, d * d)
    check(lb, P, X, N)


@pytest.mark.parametrize("n", [1, 16, 40, 64, 96])
def test_q31_shapes_and_saturation(lb, n):
    """Every tile count, with a non-contractive P that drives values into
    saturation within a few steps (codes -2^31 and 2^31 - 1, negated
    -Im P codes reaching 2^31)."""
    g = np.random.default_rng(31 + n)
    P = 1.7 * np.eye(n) + 0.2 * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))
    P[0, 0] = -1.0 - 1.0j  # a code of exactly -2^31 in both parts
    X = 0.3 * (g.standard_normal((19, n)) + 1j * g.standard_normal((19, n)))
    got = check(lb, P, X, 30)
    r, i = codes(T(got))
    assert (np.abs(r) >= 2 ** 31 - 1).any() or (np.abs(i) >= 2 ** 31 - 1).any()


def test_q15_on_the_int8_cores_matches_the_vector_kernels(lb):
    """LB_Q15 through the INT8-core kernel (variant 1400) at d = 9, B = 4096
    equals the per-row matvec bit for bit (both are the oracle's integers)."""
    H, Lk = W.transmon_system(2)
    P = T(oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS))
    X = T(W.wishart_batch(9, 4096, 7).reshape(4096, 81))
    a, b = X.clone(), X.clone()
    lb.propagate_variant(P, a, 50, 1400, "q15")
    lb.propagate_variant(P, b, 50, 901, "q15")
    assert torch.equal(a, b)


def test_q31_limits(lb):
    x = T(np.ones((2, 97), dtype=complex))
    with pytest.raises(lb.LindbladError) as e:
        lb.propagate(T(np.eye(97, dtype=complex)), x, 1, "q31")
    assert e.value.status == lb.ENOTSUP
    x = T(np.ones((2, 9), dtype=complex) * 0.1)
    x0 = x.clone()
    lb.propagate(T(np.eye(9, dtype=complex)), x, 0, "q31")
    assert torch.equal(x, x0)
