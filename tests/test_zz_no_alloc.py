"""lgt_dslash_noalloc (no context, no device allocation, library-held scratch)
against lgt_dslash, through the C ABI: two calls in a row on the same GPU,
the second on a smaller lattice, so the second reuses the scratch the first
filled; both must equal the context path bit for bit (same kernels, same
order) and the oracle to 1e-13."""
import sys

import numpy as np
import pytest

import lgt_inputs as li
from oracle import dirac

from gpu_common import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lgt():
    import torch
    assert torch.cuda.is_available()
    import paper_2602_20516_amd as m
    return m


@pytest.mark.parametrize("dagger", [False, True])
def test_noalloc_matches_context_dslash(lgt, dagger, margin):
    import torch
    cases = [((16, 16, 16, 16), 0.3, 0.125, -1), ((6, 4, 4, 8), 0.5, 0.13, +1)]  # 16^4 first, then smaller
    for dims, eps, kappa, bc in cases:
        say("noalloc dslash", dims, "dagger", dagger, "bc", bc)
        u = li.random_links(dims, eps, 611)
        psi = li.gaussian_spinor(dims, 612)
        U, P = to_dev(u), to_dev(psi)
        out = torch.full_like(P, complex(float("nan"), 0.0))
        lgt.lgt_dslash_noalloc(dims, U, P, out, kappa, dagger, fermion_bc=bc)
        lat = lgt.Lattice(dims, fermion_bc=bc)
        ref_ctx = lat.dslash(U, P, kappa, dagger)
        got = to_host(out)
        assert np.array_equal(got, to_host(ref_ctx)), f"{dims}: differs from lgt_dslash"
        ref = (dirac.dslash_dag if dagger else dirac.dslash)(u, psi, kappa, bc=bc)
        margin(f"noalloc D vs oracle {dims} dagger {dagger}", rel_err(got, ref), 1e-13)


def test_noalloc_rejects_oversize_and_bad_geometry(lgt):
    import torch
    dims = (18, 16, 16, 16)  # 73728 sites: beyond the scratch
    z = torch.zeros((16, 16, 16, 18, 4, 3), dtype=torch.complex128, device="cuda")
    U = torch.zeros((16, 16, 16, 18, 4, 3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(lgt.LGTError) as e:
        lgt.lgt_dslash_noalloc(dims, U, z, z.clone(), 0.1)
    assert "too large" in str(e.value)
    with pytest.raises(lgt.LGTError):
        lgt.lgt_dslash_noalloc((4, 4, 4, 4), U[:4, :4, :4, :4].contiguous(), z[:4, :4, :4, :4].contiguous(),
                               z[:4, :4, :4, :4].contiguous(), 0.1, fermion_bc=0)
