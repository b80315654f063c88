"""GRAPE gradient through the C-ABI against the oracle's block-triangular
Frechet gradient, central finite differences, torch.autograd.gradcheck and a
commuting-control closed form."""
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


def setup(q, M, seed_u=None):
    p = W.grape_problem(q, M=M)
    L0 = oracle.liouvillian(p["H0"], p["Lk"])
    Lc = np.stack([oracle.liouvillian(h, p["Lk"][:0]) for h in p["Hc"]])
    if seed_u is not None:
        p["u"] = np.random.default_rng(seed_u).uniform(-W.U_MAX, W.U_MAX, size=p["u"].shape)
    return p, L0, Lc


def gpu_grad(lb, p, L0, Lc, u=None, **kw):
    u = p["u"] if u is None else u
    F, g = lb.grape_gradient(T(L0), T(Lc), T(u), p["dt"], T(p["rho0"].reshape(-1)), T(p["target"].reshape(-1)), **kw)
    return F, g.cpu().numpy()


def test_grape_d3_against_oracle(lb):
    p, L0, Lc = setup(1, M=6)
    F, g = gpu_grad(lb, p, L0, Lc)
    Fo, go = oracle.grape(L0, Lc, p["u"], p["dt"], p["rho0"].reshape(-1), p["target"].reshape(-1))
    assert abs(F - Fo) < 1e-13
    assert np.abs(g - go).max() <= 1e-10 * np.abs(go).max()


def test_grape_d9_config4_sampled_slices(lb):
    """Config 4 at d = 9: M = 200 slices of 1 ns, 4 controls.  F against the
    oracle's forward pass; gradient rows of 4 seeded slices against the
    oracle's block-triangular Frechet gradient (the rest by FD below)."""
    p, L0, Lc = setup(2, M=200)
    F, g = gpu_grad(lb, p, L0, Lc)
    rows = [0, 57, 131, 199]
    Fo, go = oracle.grape(L0, Lc, p["u"], p["dt"], p["rho0"].reshape(-1), p["target"].reshape(-1), slices=rows)
    assert abs(F - Fo) < 1e-12
    scale = np.abs(go[rows]).max()
    assert np.abs(g[rows] - go[rows]).max() <= 1e-10 * scale
    assert np.all(np.isfinite(g))


def test_grape_d9_central_differences(lb):
    p, L0, Lc = setup(2, M=200)
    F, g = gpu_grad(lb, p, L0, Lc)
    h = 1e-6
    rng = np.random.default_rng(5)
    for m, c in [(0, 0), (100, 3), (199, 1)]:
        up, um = p["u"].copy(), p["u"].copy()
        up[m, c] += h
        um[m, c] -= h
        fd = (gpu_grad(lb, p, L0, Lc, up)[0] - gpu_grad(lb, p, L0, Lc, um)[0]) / (2 * h)
        assert abs(g[m, c] - fd) <= 1e-8 + 1e-7 * abs(g[m, c])
    v = rng.standard_normal(p["u"].shape)
    v /= np.linalg.norm(v)
    fd = (gpu_grad(lb, p, L0, Lc, p["u"] + h * v)[0] - gpu_grad(lb, p, L0, Lc, p["u"] - h * v)[0]) / (2 * h)
    dd = float(np.sum(g * v))
    assert abs(dd - fd) <= 1e-8 + 1e-7 * abs(dd)


def test_grape_checkpoint_recompute_matches(lb):
    """Nothing kept (checkpoint budget 1 byte): propagators rebuilt per chunk
    and the dense derivative, against the kept products and the low-rank
    derivative: the same forward pass bitwise, gradients to rounding."""
    p, L0, Lc = setup(2, M=37)
    F1, g1 = gpu_grad(lb, p, L0, Lc)
    F2, g2 = gpu_grad(lb, p, L0, Lc, checkpoint_bytes=1)
    assert F1 == F2
    assert np.abs(g1 - g2).max() <= 1e-12 * np.abs(g2).max()


def test_grape_commuting_controls_closed_form(lb):
    d = 3
    n_op = np.diag([0.0, 1.0, 2.0]).astype(complex)
    H0 = np.diag([0.0, 0.7, 1.1]).astype(complex)
    Lk = (np.sqrt(0.01) * n_op)[None]
    L0 = oracle.liouvillian(H0, Lk)
    Lc = oracle.liouvillian(n_op, Lk[:0])[None]
    M, dt = 4, 0.5
    u = np.array([[0.1], [-0.2], [0.05], [0.3]])
    rho0 = W.pure_state(d, np.random.default_rng(8))
    tgt = W.pure_state(d, np.random.default_rng(9))
    F, g = lb.grape_gradient(T(L0), T(Lc), T(u), dt, T(rho0.reshape(-1)), T(tgt.reshape(-1)))
    g = g.cpu().numpy()
    xM = oracle.expm(dt * (M * L0 + u.sum() * Lc[0])) @ rho0.reshape(-1)
    assert abs(F - np.vdot(tgt.reshape(-1), xM).real) < 1e-13
    assert np.abs(g[:, 0] - np.vdot(tgt.reshape(-1), dt * Lc[0] @ xM).real).max() < 1e-13


def test_grape_autograd_gradcheck(lb):
    p, L0, Lc = setup(1, M=3)
    L0t, Lct = T(L0), T(Lc)
    x0, w = T(p["rho0"].reshape(-1)), T(p["target"].reshape(-1))
    u = T(p["u"]).requires_grad_(True)

    def f(uu):
        return lb.GrapeFidelity.apply(uu, L0t, Lct, p["dt"], x0, w)

    assert torch.autograd.gradcheck(f, (u,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_grape_d27_directional_fd_and_forward(lb):
    """d = 27, 6 controls, M = 4 slices: F against the oracle's forward pass;
    the adjoint against a central difference along a random direction."""
    p, L0, Lc = setup(3, M=4)
    F, g = gpu_grad(lb, p, L0, Lc)
    Fo, _ = oracle.grape(L0, Lc, p["u"], p["dt"], p["rho0"].reshape(-1), p["target"].reshape(-1), want_grad=False)
    assert abs(F - Fo) < 1e-12
    h = 1e-6
    v = np.random.default_rng(3).standard_normal(p["u"].shape)
    v /= np.linalg.norm(v)
    fd = (gpu_grad(lb, p, L0, Lc, p["u"] + h * v)[0] - gpu_grad(lb, p, L0, Lc, p["u"] - h * v)[0]) / (2 * h)
    dd = float(np.sum(g * v))
    assert abs(dd - fd) <= 1e-8 + 1e-7 * abs(dd)


def test_grape_d27_lowrank_derivative_matches_dense(lb):
    """d = 27 with the build's products kept runs the Frechet derivative on
    low-rank factors (the direction x lambda^dag has rank one); with nothing
    kept (checkpoint budget 1 byte) it runs the dense recurrences.  The
    forward pass is the same build, so F is bitwise equal; the gradients
    differ only by rounding."""
    p, L0, Lc = setup(3, M=6, seed_u=5)
    F1, g1 = gpu_grad(lb, p, L0, Lc)
    F2, g2 = gpu_grad(lb, p, L0, Lc, checkpoint_bytes=1)
    assert F1 == F2
    assert np.abs(g1 - g2).max() <= 1e-11 * np.abs(g2).max()


def test_grape_chunking_does_not_change_bits(lb):
    """A workspace with a small cap forces the slices into several chunks (the
    forward builds, the backward rebuilds and the batched Frechet derivatives
    then cross chunk boundaries).  With the build's products kept (the
    default, and a 70 MB cap: all 37 slices kept, chunks of 13) the
    derivative runs on low-rank factors; under a 48 MB cap they are not kept
    and it runs dense, with and without kept propagators.  Within each kind
    the fidelity and every gradient entry are bitwise those of its
    single-chunk run; across kinds the forward pass is bitwise the same."""
    p, L0, Lc = setup(2, M=37, seed_u=21)
    F1, g1 = gpu_grad(lb, p, L0, Lc)
    Fd, gd = gpu_grad(lb, p, L0, Lc, checkpoint_bytes=1)  # dense derivative, one chunk
    assert F1 == Fd
    for cap, ckpt, ref in ((48 << 20, 0, gd), (48 << 20, 1, gd), (70 << 20, 0, g1)):
        small = lb.Workspace(cap)
        F2, g2 = gpu_grad(lb, p, L0, Lc, ws=small, checkpoint_bytes=ckpt)
        small.close()
        assert F1 == F2
        assert np.array_equal(ref, g2)


def _golden_grape(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    M, F, rows = None, None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# M "):
                M = int(line.split()[2])
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("F "):
                F = float(line.split()[1])
            else:
                m, c, v = line.split()
                rows.append((int(m), int(c), float(v)))
    return M, F, rows


@pytest.mark.parametrize("golden", ["grape_d27_M2.txt", "grape_d27_M200_sampled.txt"])
@pytest.mark.parametrize("mode", ["lowrank", "dense"])
def test_grape_d27_against_oracle_golden(lb, golden, mode):
    """Config 4 at d = 27 (6 controls, slices of 1 ns) against the oracle's
    block-triangular Frechet gradient, stored by tests/golden/make_grape_d27.py
    (M = 2: every entry; M = 200: every control of slices 0 and 199).  The
    default path (build products kept, low-rank derivative) and the dense
    recurrences (nothing kept) both within 1e-10 of the largest entry; F to
    1e-12."""
    import os
    if not os.path.exists(os.path.join(os.path.dirname(__file__), "golden", golden)):
        pytest.skip(f"{golden} not generated")
    M, Fo, rows = _golden_grape(golden)
    p, L0, Lc = setup(3, M=M)
    kw = {} if mode == "lowrank" else {"checkpoint_bytes": 1}
    F, g = gpu_grad(lb, p, L0, Lc, **kw)
    assert abs(F - Fo) < 1e-12
    go = np.array([v for _, _, v in rows])
    gg = np.array([g[m, c] for m, c, _ in rows])
    assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max(), (np.abs(gg - go).max(), np.abs(go).max())
    assert np.all(np.isfinite(g))
