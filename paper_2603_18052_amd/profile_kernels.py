"""Workload for rocprofv3 counter runs: one plain device copy of a known
size (calibrates FETCH_SIZE / WRITE_SIZE against bytes actually moved), then
one chain on the d = 9 workload (B = 4096 Wishart states, 1e4 steps) or the
d = 27 workload (--d 27: B = 1024, a few steps) in the requested precision,
or (--grape) one GRAPE gradient of the M = 200 slice workload at that d.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- \\
        python -m paper_2603_18052_amd.profile_kernels --precision c128
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 512 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="c128")
    ap.add_argument("--d", type=int, default=9, choices=(9, 27))
    ap.add_argument("--nsteps", type=int, default=None, help="default 10^4 (d = 9), 40 (d = 27)")
    ap.add_argument("--batch", default=None,
                    help="default 4096 (d = 9), 1024 (d = 27); a comma list runs each batch in turn")
    ap.add_argument("--variant", default=None,
                    help="chain variant(s) to launch (comma list, each in turn); default: the library's choice")
    ap.add_argument("--grape", action="store_true", help="one GRAPE gradient (M = 200) instead of a chain")
    a = ap.parse_args()
    if a.nsteps is None:
        a.nsteps = 10_000 if a.d == 9 else 40
    batches = [4096 if a.d == 9 else 1024] if a.batch is None else [int(b) for b in str(a.batch).split(",")]
    variants = [None] if a.variant is None else [int(v) for v in a.variant.split(",")]
    import torch
    from paper_2603_18052_amd import lindblad as lb
    from paper_2603_18052_amd import workloads as W

    dev = torch.device("cuda:0")
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)  # the calibration copy: COPY_BYTES read, COPY_BYTES written
    torch.cuda.synchronize()
    if a.grape:
        p = W.grape_problem(2 if a.d == 9 else 3, M=200)
        Hc = torch.from_numpy(p["Hc"]).to(dev)
        L0 = lb.liouvillian(torch.from_numpy(p["H0"]).to(dev), torch.from_numpy(p["Lk"]).to(dev))
        Lc = torch.stack([lb.liouvillian(Hc[c], None) for c in range(Hc.shape[0])])
        x0 = torch.from_numpy(p["rho0"].reshape(-1)).to(dev)
        w = torch.from_numpy(p["target"].reshape(-1)).to(dev)
        F, g = lb.grape_gradient(L0, Lc, torch.from_numpy(p["u"]).to(dev), p["dt"], x0, w)
        torch.cuda.synchronize()
        print("profile_kernels: done grape", a.d, F, flush=True)
        return
    cfg = (W.config2 if a.d == 9 else W.config3)(B=max(batches), nsteps=a.nsteps)
    H, Lk = torch.from_numpy(cfg["H"]).to(dev), torch.from_numpy(cfg["Lk"]).to(dev)
    P = lb.propagator(lb.liouvillian(H, Lk), cfg["dt"])
    X0 = torch.from_numpy(cfg["rho0"].reshape(max(batches), -1)).to(dev)
    for B in batches:
        for v in variants:
            X = X0[:B].clone()
            torch.cuda.synchronize()
            if a.precision == "baseline":
                lb.propagate_baseline(P, X, a.nsteps)
            elif v is None:
                lb.propagate(P, X, a.nsteps, a.precision)
            else:
                lb.propagate_variant(P, X, a.nsteps, v, a.precision)
            torch.cuda.synchronize()
            print("profile_kernels: done", a.precision, "B", B, "variant", v, flush=True)


if __name__ == "__main__":
    main()
