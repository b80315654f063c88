"""The C ABI from plain C: tests/c/abi_client.c is compiled with gcc against
include/lindblad.h and liblindblad.so (no Python, no torch in the client),
run as a child process on inputs written here, and its L, P and final states
are checked against the oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2603_18052_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_18052_amd")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    from paper_2603_18052_amd import lindblad
    lindblad.lib()  # the library is built
    exe = str(tmp_path_factory.mktemp("cclient") / "abi_client")
    cmd = ["gcc", "-O2", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c", "abi_client.c"), "-o", exe,
           "-L", PKG, "-llindblad", "-L", "/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{PKG}",
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("q,B,N,variant", [(1, 3, 500, 301), (2, 20, 200, 502)])
def test_c_client_matches_oracle(client, tmp_path, q, B, N, variant):
    d = 3 ** q
    H, Lk = W.transmon_system(q)
    X = W.wishart_batch(d, B, 40 + q).reshape(B, d * d)
    np.ascontiguousarray(H, dtype=np.complex128).tofile(tmp_path / "H.bin")
    np.ascontiguousarray(Lk, dtype=np.complex128).tofile(tmp_path / "Lk.bin")
    np.ascontiguousarray(X, dtype=np.complex128).tofile(tmp_path / "rho.bin")
    r = subprocess.run([client, str(tmp_path), str(d), str(Lk.shape[0]), str(B), str(N), repr(W.DT_NS), str(variant)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    n = d * d
    L = np.fromfile(tmp_path / "L.bin", dtype=np.complex128).reshape(n, n)
    P = np.fromfile(tmp_path / "P.bin", dtype=np.complex128).reshape(n, n)
    out = np.fromfile(tmp_path / "rho_out.bin", dtype=np.complex128).reshape(B, n)
    outv = np.fromfile(tmp_path / "rho_variant.bin", dtype=np.complex128).reshape(B, n)
    s_used, chosen = map(int, (tmp_path / "s.txt").read_text().split())
    Lref = oracle.liouvillian(H, Lk)
    assert np.abs(L - Lref).max() <= 1e-14 * np.abs(Lref).max()
    Pref, sref = oracle.expm(Lref * W.DT_NS, return_s=True)
    assert s_used == sref
    assert oracle.rel_fro(P, Pref) < 1e-12
    ref = oracle.propagate(P, X, N)  # chain parity from the same P
    assert oracle.rel_per_state(out, ref) < 1e-12
    assert oracle.rel_per_state(outv, ref) < 1e-12
    assert chosen > 0
