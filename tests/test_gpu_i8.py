"""GPU parity of the INT8-digit chain (LB_I8_SLICED) against the CPU oracle.

The sliced INT8 step is exact integer arithmetic on digits of P and of the
state, so its error against the FP64 oracle chain comes only from the
representation: P rounded to 38 bits below its row's power of two, the state
to 30 bits below its own, levels above 4 dropped.  One step is within
~1e-9 of P x for states of norm ~1; the configurations' chains stay below
the 1e-6 trace-distance target (reading: "split precision on MFMA", the
sliced form that meets the bound).
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


def run(lb, P, X, nsteps):
    x = T(X.copy())
    lb.propagate(T(P), x, nsteps, "i8_sliced")
    return x.cpu().numpy()


def test_i8_single_step(lb, P9):
    """One step against P x: the error of 30-bit state and 38-bit row-scaled
    P digits, ~2^-31 of the state's largest entry per output."""
    X = states(9, 16, 3)
    got = run(lb, P9, X, 1)
    err = np.abs(got - X @ P9.T).max()
    print(f"i8 one step: max abs error {err:.3e}")
    assert err < 2e-9


@pytest.mark.parametrize("nsteps", [1000, 10000])
def test_i8_d9_meets_1e6(lb, P9, nsteps):
    X = states(9, 37, 41)  # two full workgroups and a ragged one
    ref = oracle.propagate(P9, X, nsteps)
    got = run(lb, P9, X, nsteps)
    td = oracle.trace_distance(got.reshape(-1, 9, 9), ref.reshape(-1, 9, 9))
    print(f"i8 d=9 N={nsteps}: trace distance max {td.max():.3e} median {np.median(td):.3e}")
    assert td.max() < 1e-6
    rep = oracle.state_report(got.reshape(-1, 9, 9))
    assert rep["trace_err"].max() < 1e-6 and rep["lambda_min"].min() > -1e-6


def test_i8_d3_config1(lb, P3):
    c = W.config1()
    ref = oracle.propagate(P3, c["rho0"].reshape(1, 9), c["nsteps"])
    got = run(lb, P3, c["rho0"].reshape(1, 9), c["nsteps"])
    td = oracle.trace_distance(got.reshape(3, 3), ref.reshape(3, 3))
    print(f"i8 d=3 N=1e4: trace distance {td:.3e}")
    assert td < 1e-6


@pytest.mark.parametrize("n", [1, 9, 16, 40, 64, 81, 85, 96])
def test_i8_shapes(lb, n):
    """Every tile count (1 .. 12 row tiles of the 2n real embedding, 1 .. 3
    k chunks) on a random contraction, 19 states (a ragged workgroup).  The
    states shrink by up to 1e-12 over 40 steps, so the error is taken
    relative to each state's initial norm."""
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    P = A / (1.02 * np.linalg.norm(A, 2))
    X = g.standard_normal((19, n)) + 1j * g.standard_normal((19, n))
    ref = oracle.propagate(P, X, 40)
    got = run(lb, P, X, 40)
    assert oracle.rel_per_state(got, ref, X) < 1e-8


def test_i8_deterministic_zero_state_and_chunked_calls(lb, P9):
    """Bitwise repeatable; a zero state stays zero; 1000 steps as ten calls
    of 100 stay within the bound of one call (a call slices its first state
    below that state's own exponent; inside a call the next state is sliced
    below the previous state's exponent unless it outgrew the top digit's
    headroom, so the bits may differ at call boundaries)."""
    X = states(9, 20, 5)
    X[7] = 0.0
    a = run(lb, P9, X, 1000)
    b = run(lb, P9, X, 1000)
    assert np.array_equal(a, b)
    assert not a[7].any()
    x = T(X.copy())
    for _ in range(10):
        lb.propagate(T(P9), x, 100, "i8_sliced")
    ref = oracle.propagate(P9, X, 1000)
    keep = np.arange(20) != 7
    td = oracle.trace_distance(x.cpu().numpy()[keep].reshape(-1, 9, 9), ref[keep].reshape(-1, 9, 9))
    assert td.max() < 1e-6
    x = T(X.copy())
    lb.propagate(T(P9), x, 0, "i8_sliced")
    assert np.array_equal(x.cpu().numpy(), X)


@pytest.mark.parametrize("n", [1, 9, 40, 64, 81, 96])
def test_i8_fused_forms_agree_bitwise(lb, n):
    """Eight wavefronts (1300: up to two row tiles each) and four (1301: up
    to three) with a barrier per step, and eight with pipelined steps (1302:
    per-tile progress words, three digit buffers) run the same arithmetic on
    the same digits, so they give the same bits; a growing propagator makes
    every step re-slice (the pipelined form redoes the step's first tile)."""
    g = np.random.default_rng(100 + n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    P = A / (1.02 * np.linalg.norm(A, 2))
    X = g.standard_normal((37, n)) + 1j * g.standard_normal((37, n))
    for Pm, steps in ((P, 50), (3.0 * np.eye(n, dtype=complex) + 0.01 * A, 20)):
        out = {}
        for v in (1300, 1301, 1302):
            x = T(X.copy())
            lb.propagate_variant(T(Pm), x, steps, v, "i8_sliced")
            out[v] = x.cpu().numpy()
        for v in (1301, 1302):
            assert np.array_equal(out[1300], out[v]), v
        ref = oracle.propagate(Pm, X, steps)
        assert oracle.rel_per_state(out[1302], ref, X) < 1e-8


def test_i8_growing_states_take_the_exact_exponent(lb):
    """A propagator that quadruples the state every step (4 I): every step
    grows past the top digit's headroom, so every step takes the re-slicing
    path; one that doubles it (2 I) and one that grows it by 1.6 cross a
    power of two every step or two and stay within the headroom (31-bit
    digits until the next step's exponent catches up).  The results stay
    within the representation's bound."""
    X = states(9, 5, 9)
    got = run(lb, 4.0 * np.eye(81, dtype=complex), X, 12)
    assert oracle.rel_per_state(got, X * 4.0 ** 12) < 1e-8
    got = run(lb, 2.0 * np.eye(81, dtype=complex), X, 20)
    assert oracle.rel_per_state(got, X * 2.0 ** 20) < 1e-8
    P = 1.6 * np.eye(81, dtype=complex)
    P[0, 1] = 0.01
    ref = oracle.propagate(P, X, 30)
    got = run(lb, P, X, 30)
    # each step rounds the state to 2^-30 of its largest entry: N 2^-30 relative
    assert oracle.rel_per_state(got, ref) < 30 * 2.0 ** -30


def test_i8_config2_fused_forms_full_size_bitwise(lb, P9):
    """The bench's configuration (4096 Wishart states, 1e4 steps) in each
    fused form the tuner may pick: the barrier forms (1300, 1301) and the
    pipelined one (1302) give the same bits at full size."""
    c = W.config2()
    X = c["rho0"].reshape(-1, 81)
    out = {}
    for v in (1300, 1301, 1302):
        x = T(X.copy())
        lb.propagate_variant(T(P9), x, c["nsteps"], v, "i8_sliced")
        out[v] = x.cpu().numpy()
    assert np.array_equal(out[1300], out[1301])
    assert np.array_equal(out[1300], out[1302])


def test_i8_config2_full_size_sampled(lb, P9):
    """The configuration the bench times: 4096 Wishart states, 1e4 steps, on
    the oracle's P; sampled states against the oracle's chain."""
    c = W.config2()
    X = c["rho0"].reshape(-1, 81)
    idx = np.array([0, 1, 15, 16, 777, 2048, 4094, 4095])
    ref = oracle.propagate(P9, X[idx], c["nsteps"])
    x = T(X.copy())
    lb.propagate(T(P9), x, c["nsteps"], "i8_sliced")
    got = x.cpu().numpy()[idx]
    td = oracle.trace_distance(got.reshape(-1, 9, 9), ref.reshape(-1, 9, 9))
    print(f"i8 config 2 (B=4096, N=1e4) sampled: trace distance max {td.max():.3e}")
    assert td.max() < 1e-6


# ------------------------------------------------ per-step GEMM (n > 96)
@pytest.fixture(scope="module")
def P27():
    H, Lk = W.transmon_system(3)
    return oracle.propagator(oracle.liouvillian(H, Lk), W.DT_NS)


def test_i8_gemm_d27_config3(lb, P27):
    """Config 3 (d = 27, 10^3 steps) on the oracle's P: a ragged batch, the
    trace distance against the oracle's chain."""
    X = states(27, 37, 17)
    ref = oracle.propagate(P27, X, 1000)
    got = run(lb, P27, X, 1000)
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"i8 GEMM d=27 B=37 N=1e3: trace distance max {td.max():.3e} median {np.median(td):.3e}")
    assert td.max() < 1e-6
    rep = oracle.state_report(got.reshape(-1, 27, 27))
    assert rep["trace_err"].max() < 1e-6 and rep["lambda_min"].min() > -1e-6


@pytest.mark.parametrize("B", [1, 512, 1024])
def test_i8_gemm_d27_full_batch_sampled(lb, P27, B):
    c = W.config3(B=B)
    X = c["rho0"].reshape(-1, 729)
    idx = np.unique(np.array([0, 1, 63, 64, 700, 1023]) % B)
    ref = oracle.propagate(P27, X[idx], c["nsteps"])
    x = T(X.copy())
    lb.propagate(T(P27), x, c["nsteps"], "i8_sliced")
    got = x.cpu().numpy()[idx]
    td = oracle.trace_distance(got.reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    print(f"i8 GEMM config 3 B={B} sampled: trace distance max {td.max():.3e}")
    assert td.max() < 1e-6


@pytest.mark.parametrize("variant", [1500, 1501, 1502, 1503])
@pytest.mark.parametrize("n", [97, 100, 130, 260])
def test_i8_gemm_shapes(lb, n, variant):
    """The four tile shapes (1500: 96 rows x 64 states, 1501: 96 x 32 with
    four ring slots, 1502: 64 x 16 with six, 1503: 96 x 32 with two, two
    workgroups per CU), 64-deep k chunks and ragged state tiles (B = 19) on
    random contractions (relative to each state's initial norm: the states
    shrink by orders of magnitude); n = 260 has k padding that no row block
    covers."""
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    P = A / (1.02 * np.linalg.norm(A, 2))
    X = g.standard_normal((19, n)) + 1j * g.standard_normal((19, n))
    ref = oracle.propagate(P, X, 30)
    x = T(X.copy())
    lb.propagate_variant(T(P), x, 30, variant, "i8_sliced")
    assert oracle.rel_per_state(x.cpu().numpy(), ref, X) < 1e-8


@pytest.mark.parametrize("B", [1, 19, 64, 129])
def test_i8_gemm_tile_shapes_agree_bitwise(lb, P27, B):
    """The digit sums are exact integers and the epilogue's arithmetic does
    not depend on the tiling, so the four tile shapes (and the small
    shape's graph-replayed twin, 1552) give the same bits; the result meets
    the 1e-6 bound against the oracle."""
    X = states(27, B, 31 + B)
    out = {}
    for v in (1500, 1501, 1502, 1503, 1552):
        x = T(X.copy())
        lb.propagate_variant(T(P27), x, 60, v, "i8_sliced")
        out[v] = x.cpu().numpy()
    for v in (1501, 1502, 1503, 1552):
        assert np.array_equal(out[1500], out[v]), v
    idx = np.unique(np.array([0, B // 2, B - 1]))
    ref = oracle.propagate(P27, X[idx], 60)
    td = oracle.trace_distance(out[1502][idx].reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    assert td.max() < 1e-6


def test_i8_gemm_graph_twin_deterministic_and_chunked(lb, P27):
    """The graph-replayed twin (1550) equals the direct launches (1500) bit
    for bit, runs repeat bitwise, and a run split into calls stays within
    the bound (each call restarts from the exact exponent, so the bits may
    differ from one long call)."""
    X = states(27, 20, 23)
    out = {}
    for v in (1500, 1550):
        x = T(X.copy())
        lb.propagate_variant(T(P27), x, 100, v, "i8_sliced")
        out[v] = x.cpu().numpy()
    assert np.array_equal(out[1500], out[1550])
    x = T(X.copy())
    lb.propagate_variant(T(P27), x, 100, 1500, "i8_sliced")
    assert np.array_equal(x.cpu().numpy(), out[1500])
    x = T(X.copy())
    for _ in range(4):
        lb.propagate(T(P27), x, 25, "i8_sliced")
    ref = oracle.propagate(P27, X, 100)
    td = oracle.trace_distance(x.cpu().numpy().reshape(-1, 27, 27), ref.reshape(-1, 27, 27))
    assert td.max() < 1e-6
