"""The allocation-free probe entry point (coil_field_at_noalloc, scratch in a
static device array) against coil_field_at on the same handle: two calls in a
row, the second with fewer points, FP64 agreement to 1e-10 normwise."""
import numpy as np
import pytest

import coil_synth as cs

pytestmark = pytest.mark.gpu


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def test_field_at_noalloc_matches_field_at():
    import torch
    import paper_2403_07666_amd as pk
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    g = pk.Coil(w, inp)
    g.run(150)  # non-trivial currents
    rng = np.random.Generator(np.random.PCG64(21))
    for npts in (5000, 333):
        r = np.concatenate([[0.0], rng.uniform(0.0, 0.08, npts - 1)])
        z = rng.uniform(-0.02, 0.02, npts)
        br_ref, bz_ref = g.field_at(r, z)
        dev = g.device
        rd = torch.from_numpy(r).to(dev)
        zd = torch.from_numpy(z).to(dev)
        brd = torch.full((npts,), np.nan, dtype=torch.float64, device=dev)
        bzd = torch.full((npts,), np.nan, dtype=torch.float64, device=dev)
        torch.cuda.synchronize(dev)
        g.field_at_noalloc(rd, zd, brd, bzd)
        g.synchronize()
        br, bz = brd.cpu().numpy(), bzd.cpu().numpy()
        assert np.all(np.isfinite(br)) and np.all(np.isfinite(bz))
        assert br[0] == 0.0  # on the axis
        e = max(nerr(br, br_ref), nerr(bz, bz_ref))
        print(f"npts {npts}: {e:.2e}", flush=True)
        assert e <= 1e-10
    # beyond the static scratch: a clear error, nothing launched
    big = pk.FIELD_AT_SCRATCH_BYTES // 16 + 1
    assert pk.lib().coil_field_at_noalloc(g.h, big, None, None, None, None) == -1
    assert b"exceeds" in pk.lib().coil_last_error()
