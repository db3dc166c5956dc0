"""Launch the even/odd hop kernel and a plain 512 MB device copy, for
rocprofv3 kernel traces and FETCH_SIZE / WRITE_SIZE counter passes.

Usage: python paper_2602_20516_amd/hop_probe.py [Lx Ly Lz Lt] [fp64|mixed_fp32] [nrhs]
(nrhs > 1 times the batched hop over nrhs right-hand sides instead)
The copy (torch's copy kernel, 512 MiB read + 512 MiB written) calibrates the
counters: bytes per hop launch = counter(hop) / counter(copy) * 512 MiB.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))  # repository root
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import lgt_inputs as li  # noqa: E402
import paper_2602_20516_amd as lgt  # noqa: E402


def main():
    dims = tuple(int(v) for v in sys.argv[1:5]) if len(sys.argv) >= 5 else (16, 16, 16, 16)
    prec = sys.argv[5] if len(sys.argv) >= 6 else "fp64"
    u = li.random_links(dims, 0.3, 201)
    eta = li.gaussian_spinor(dims, 202)
    U = torch.from_numpy(u).to("cuda")
    E = torch.from_numpy(eta).to("cuda")
    nrhs = int(sys.argv[6]) if len(sys.argv) >= 7 else 1
    lat = lgt.Lattice(dims)
    ms = lat.hop_benchmark_mrhs(U, E, nrhs, prec, 20) if nrhs > 1 else lat.hop_benchmark(U, E, prec, 20)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"hop {dims} {prec} nrhs {nrhs}: {ms * 1e3:.2f} us per launch; copy of {a.numel() * 8 >> 20} MiB x5 done",
          flush=True)


if __name__ == "__main__":
    main()
