"""Fixed-point chain (LB_Q15, Alg. 5): every variant bit-exact against the
oracle's integer chain (integer sums do not depend on their order), on the
paper's d = 3 drift model over its step counts, on transmon propagators at
d = 9 and 27, and with saturation forced."""
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
    """Q1.15 codes of the GPU result (its values are integers / 2^15 exactly)."""
    x = x.cpu().numpy()
    re, im = np.rint(x.real * 32768), np.rint(x.imag * 32768)
    assert np.array_equal(re / 32768, x.real) and np.array_equal(im / 32768, x.imag)
    return re.astype(np.int64), im.astype(np.int64)


def check_all_variants(lb, P, X, N):
    n = P.shape[0]
    ref_r, ref_i = oracle.propagate_q15(P, X, N)
    variants = lb.chain_variants(n, "q15", X.shape[0])
    assert variants
    for v in variants:
        x = T(X.copy())
        lb.propagate_variant(T(P), x, N, v, "q15")
        r, i = codes(x)
        assert np.array_equal(r, ref_r.reshape(r.shape)) and np.array_equal(i, ref_i.reshape(i.shape)), \
            (lb.variant_name(v), N)


@pytest.mark.parametrize("drive", [0.0, 0.05])
@pytest.mark.parametrize("N", [1, 10, 100, 1000, 10000])
def test_q15_paper_drift_model(lb, drive, N):
    H, Lk, dt, rho0 = W.paper_fixed_point_model(drive)
    P = oracle.propagator(oracle.liouvillian(H, Lk), dt)
    check_all_variants(lb, P, rho0.reshape(1, 9), N)


@pytest.mark.parametrize("q,B,N", [(1, 37, 500), (2, 20, 300), (3, 3, 70)])
def test_q15_transmon_chains(lb, q, B, N):
    d = 3 ** q
    H, Lk = W.transmon_system(q)
    P = oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)
    X = W.wishart_batch(d, B, 60 + q).reshape(B, d * d)
    check_all_variants(lb, P, X, N)


def test_q15_saturation(lb):
    """A non-contractive P drives values into saturation within a few steps."""
    g = np.random.default_rng(15)
    P = 1.7 * np.eye(16) + 0.2 * (g.standard_normal((16, 16)) + 1j * g.standard_normal((16, 16)))
    X = 0.3 * (g.standard_normal((5, 16)) + 1j * g.standard_normal((5, 16)))
    check_all_variants(lb, P, X, 40)
    x = T(X.copy())
    lb.propagate(T(P), x, 40, "q15")
    r, i = codes(x)
    assert (np.abs(r) == 32768).any() or (r == 32767).any() or (np.abs(i) == 32768).any() or (i == 32767).any()
