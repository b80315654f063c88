"""Seeded synthetic inputs for dense Lindblad propagation (numpy only).

This module builds the *inputs* of the method: Hamiltonians, collapse
operators, control Hamiltonians, control amplitudes, initial states and
targets.  It contains none of the method's own arithmetic (no superoperator
assembly, no exponential, no propagation); both the CPU oracle and the GPU
path consume what it returns.

Physical model (units: hbar = 1, time in ns, angular frequency in rad/ns):

* A transmon is truncated to 3 levels, annihilation operator
  ``a = sum_k sqrt(k) |k-1><k|``.  With ``q`` transmons, ``d = 3**q`` and
  ``a_j = I x ... x a x ... x I`` with transmon 1 the most significant index.
* Anharmonic term ``(alpha/2) a^dag a^dag a a = diag(0, 0, alpha)`` per
  transmon, alpha = 2 pi * (-200 MHz); drive ``Omega (a + a^dag)`` with
  Omega = 2 pi * 20 MHz; exchange coupling ``g (a_j^dag a_{j+1} + h.c.)``
  between chain neighbours only, g = 2 pi * 5 MHz.
* Collapse operators, ordered per transmon: ``sqrt(gamma1) a_j`` with
  gamma1 = 1/T1, T1 = 50 us, then ``sqrt(gamma_phi) a_j^dag a_j`` with
  gamma_phi = 1/T_phi, T_phi = 60 us (the operator is taken literally, so
  the 0-1 coherence decays at gamma_phi/2).
* GRAPE: the drift omits the static drive; controls per transmon are
  ``H_x = a + a^dag`` and ``H_y = i (a^dag - a)`` ordered ``c = 2j, 2j+1``;
  amplitudes are uniform in [-2 pi * 30 MHz, 2 pi * 30 MHz].
* Random states: pure ``psi = z/|z|`` with ``z ~ CN(0, I)``; mixed
  (Wishart) ``rho = G G^dag / Tr(G G^dag)`` with ``G`` a d x r complex
  Gaussian matrix and rank r uniform in {1..d}.

Every generator draws from ``numpy.random.default_rng([260318052, config,
stream])``; stream 0 = states, 1 = controls, 2 = targets, 3 = problem shapes.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 260318052

TWO_PI = 2.0 * np.pi
ALPHA = TWO_PI * -0.200      # anharmonicity, rad/ns
OMEGA = TWO_PI * 0.020       # static drive, rad/ns
G_COUPLING = TWO_PI * 0.005  # exchange coupling, rad/ns
U_MAX = TWO_PI * 0.030       # control amplitude bound, rad/ns
T1_NS = 50_000.0
TPHI_NS = 60_000.0
GAMMA1 = 1.0 / T1_NS
GAMMA_PHI = 1.0 / TPHI_NS
DT_NS = 0.5                  # propagation step of the fixed-step configs
DT_GRAPE_NS = 1.0            # GRAPE slice length
LEVELS = 3


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(config), int(stream)])


# ---------------------------------------------------------------- operators
def annihilation(levels: int = LEVELS) -> np.ndarray:
    a = np.zeros((levels, levels), dtype=np.complex128)
    for k in range(1, levels):
        a[k - 1, k] = np.sqrt(k)
    return a


def embed(op: np.ndarray, j: int, q: int) -> np.ndarray:
    """``I x .. x op (position j, 0 = most significant) x .. x I``."""
    out = np.ones((1, 1), dtype=np.complex128)
    eye = np.eye(op.shape[0], dtype=np.complex128)
    for k in range(q):
        out = np.kron(out, op if k == j else eye)
    return out


def ladder_ops(q: int):
    a = annihilation()
    return [embed(a, j, q) for j in range(q)]


def drift_hamiltonian(q: int, static_drive: bool = True) -> np.ndarray:
    """Anharmonic terms, optional static drive, neighbour exchange."""
    aa = ladder_ops(q)
    d = LEVELS ** q
    H = np.zeros((d, d), dtype=np.complex128)
    for a in aa:
        ad = a.conj().T
        H += 0.5 * ALPHA * (ad @ ad @ a @ a)
        if static_drive:
            H += OMEGA * (a + ad)
    for j in range(q - 1):
        x = aa[j].conj().T @ aa[j + 1]
        H += G_COUPLING * (x + x.conj().T)
    return H


def collapse_ops(q: int) -> np.ndarray:
    """K = 2q operators, shape (K, d, d): [sqrt(g1) a_1, sqrt(gphi) n_1, ...]."""
    out = []
    for a in ladder_ops(q):
        out.append(np.sqrt(GAMMA1) * a)
        out.append(np.sqrt(GAMMA_PHI) * (a.conj().T @ a))
    return np.ascontiguousarray(np.stack(out))


def control_hamiltonians(q: int) -> np.ndarray:
    """C = 2q controls, shape (C, d, d): H_x = a + a^dag, H_y = i(a^dag - a)."""
    out = []
    for a in ladder_ops(q):
        ad = a.conj().T
        out.append(a + ad)
        out.append(1j * (ad - a))
    return np.ascontiguousarray(np.stack(out))


def transmon_system(q: int):
    """(H, Lk) of the fixed-step propagation configs for q transmons."""
    return drift_hamiltonian(q, static_drive=True), collapse_ops(q)


def paper_grape_model(d: int, drive: float = 0.05):
    """The paper's own landscape-point model: H0 = diag(0..d-1) plus a small
    truncated sigma_x-type drive, amplitude damping with T1 = 50 and pure
    dephasing with T2 = 30 (dimensionless units, dt = 0.5).  Used only to pin
    the scaling exponent; the dephasing rate follows 1/T2 = 1/(2 T1) + gphi."""
    a = annihilation(d)
    H = np.diag(np.arange(d, dtype=np.float64)).astype(np.complex128)
    H += drive * (a + a.conj().T)
    t1, t2 = 50.0, 30.0
    gphi = 1.0 / t2 - 0.5 / t1
    Lk = np.stack([np.sqrt(1.0 / t1) * a,
                   np.sqrt(2.0 * gphi) * (a.conj().T @ a)])
    return H, Lk, 0.5


def paper_fixed_point_model(drive: float = 0.05):
    """The paper's d = 3 fixed-point drift model (its FPGA section): H0 =
    diag(0, 1, 2) plus drive * sigma_x on the |0>-|1> pair, amplitude damping
    with T1 = 50 and dephasing sqrt(1/T2 - 1/(2 T1)) a^dag a with T2 = 30
    (dimensionless units), dt = 0.5, started from |0><0|.  Returns H, Lk, dt,
    rho0."""
    d = 3
    a = annihilation(d)
    H = np.diag(np.arange(d, dtype=np.float64)).astype(np.complex128)
    H[0, 1] += drive
    H[1, 0] += drive
    t1, t2 = 50.0, 30.0
    Lk = np.stack([np.sqrt(1.0 / t1) * a, np.sqrt(1.0 / t2 - 0.5 / t1) * (a.conj().T @ a)])
    rho0 = np.zeros((d, d), dtype=np.complex128)
    rho0[0, 0] = 1.0
    return H, Lk, 0.5, rho0


# ------------------------------------------------------------------- states
def pure_state(d: int, g: np.random.Generator) -> np.ndarray:
    z = g.standard_normal(d) + 1j * g.standard_normal(d)
    z /= np.linalg.norm(z)
    return np.outer(z, z.conj())


def pure_ket(d: int, g: np.random.Generator) -> np.ndarray:
    z = g.standard_normal(d) + 1j * g.standard_normal(d)
    return z / np.linalg.norm(z)


def wishart_state(d: int, g: np.random.Generator, rank: int | None = None) -> np.ndarray:
    r = int(g.integers(1, d + 1)) if rank is None else int(rank)
    G = g.standard_normal((d, r)) + 1j * g.standard_normal((d, r))
    rho = G @ G.conj().T
    return rho / np.trace(rho).real


def wishart_batch(d: int, B: int, config: int) -> np.ndarray:
    """B Wishart states, shape (B, d, d) complex128, rank uniform in {1..d}."""
    g = rng(config, 0)
    out = np.empty((B, d, d), dtype=np.complex128)
    for b in range(B):
        out[b] = wishart_state(d, g)
    return out


# -------------------------------------------------------------- the configs
def config1():
    """d = 3 single transmon, one Haar pure state, dt = 0.5 ns, 1e4 steps."""
    H, Lk = transmon_system(1)
    rho0 = pure_state(3, rng(1, 0))[None]
    return dict(d=3, H=H, Lk=Lk, dt=DT_NS, rho0=rho0, nsteps=10_000)


def config2(B: int = 4096, nsteps: int = 10_000):
    """d = 9 two coupled transmons, B Wishart states, dt = 0.5 ns."""
    H, Lk = transmon_system(2)
    return dict(d=9, H=H, Lk=Lk, dt=DT_NS, rho0=wishart_batch(9, B, 2), nsteps=nsteps)


def config3(B: int = 1024, nsteps: int = 1000):
    """d = 27 three-transmon chain, B Wishart states, dt = 0.5 ns."""
    H, Lk = transmon_system(3)
    return dict(d=27, H=H, Lk=Lk, dt=DT_NS, rho0=wishart_batch(27, B, 3), nsteps=nsteps)


def grape_problem(q: int, M: int = 200, config: int = 4):
    """GRAPE config: drift without static drive, 2q controls, M slices of
    1 ns, amplitudes u (M, C), rho0 = |0..0><0..0|, Haar pure target."""
    d = LEVELS ** q
    H0 = drift_hamiltonian(q, static_drive=False)
    Hc = control_hamiltonians(q)
    Lk = collapse_ops(q)
    C = Hc.shape[0]
    u = rng(config * 10 + q, 1).uniform(-U_MAX, U_MAX, size=(M, C))
    rho0 = np.zeros((d, d), dtype=np.complex128)
    rho0[0, 0] = 1.0
    target = pure_state(d, rng(config * 10 + q, 2))
    return dict(d=d, H0=H0, Hc=Hc, Lk=Lk, M=M, dt=DT_GRAPE_NS, u=u,
                rho0=rho0, target=target)


def mixed_batch(nprob: int = 256, nmin: int = 100, nmax: int = 10_000, config: int = 5):
    """Serving-style mix: problem i has d = (3, 9, 27)[i mod 3], its own
    constant x/y control amplitudes per transmon added to the drift, a
    Wishart initial state and a step count uniform in {nmin..nmax}."""
    gshape = rng(config, 3)
    gctl = rng(config, 1)
    gst = rng(config, 0)
    probs = []
    for i in range(nprob):
        q = (1, 2, 3)[i % 3]
        d = LEVELS ** q
        H = drift_hamiltonian(q, static_drive=False)
        Hc = control_hamiltonians(q)
        amps = gctl.uniform(-U_MAX, U_MAX, size=Hc.shape[0])
        H = H + np.tensordot(amps, Hc, axes=1)
        probs.append(dict(d=d, H=H, Lk=collapse_ops(q), dt=DT_NS,
                          rho0=wishart_state(d, gst),
                          nsteps=int(gshape.integers(nmin, nmax + 1))))
    return probs
