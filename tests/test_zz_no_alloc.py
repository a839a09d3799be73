"""The scalar product entry point that allocates nothing (smps_scprod_noalloc)
against smps_scprod (Sec. 2.4.4 transfer-matrix sweep) and the oracle: two
calls in a row, the second on a smaller pair, on a fresh context whose
workspace arena must stay empty; oversized inputs are refused."""

import math

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def _pair(seed, L, chi):
    rng = np.random.default_rng(seed)
    return synth.random_mps(rng, L, 2, chi), synth.random_mps(rng, L, 2, chi)


def test_scprod_noalloc_matches_scprod_and_allocates_nothing():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ctx = B.Context(0)
    try:
        cases = [_pair(11, 14, 128), _pair(12, 9, 16)]  # the second call is smaller
        handles = [(ctx.mps_create(a), ctx.mps_create(b)) for a, b in cases]
        assert ctx.workspace_bytes() == 0
        outs = []
        for ha, hb in handles:
            out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.scprod_noalloc(ha, hb, out.data_ptr())
            torch.cuda.synchronize()
            outs.append(float(out.item()))
        # nothing was allocated: the context's arena is still empty
        assert ctx.workspace_bytes() == 0
        for (a, b), (ha, hb), got in zip(cases, handles, outs):
            ref_gpu = ctx.scprod(ha, hb)
            ref_cpu = om.scprod(a, b)
            scale = math.sqrt(om.scprod(a, a) * om.scprod(b, b))
            # same products in the same order as smps_scprod: identical bits
            assert got == ref_gpu, (got, ref_gpu)
            assert abs(got - ref_cpu) <= 1e-12 * scale
        # the second (smaller) call must not see the first call's leftovers:
        # rerun the small pair after a large one and compare again
        ha, hb = handles[1]
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.scprod_noalloc(*handles[0], out.data_ptr())
        ctx.scprod_noalloc(ha, hb, out.data_ptr())
        torch.cuda.synchronize()
        assert float(out.item()) == outs[1]
        for ha, hb in handles:
            ha.destroy()
            hb.destroy()
    finally:
        ctx.close()


def test_scprod_noalloc_refuses_inputs_beyond_its_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ctx = B.Context(0)
    try:
        # chi = 512 at d = 2: two 512 x 512 transfer matrices and a 512 x 2 x 512
        # partial product need 8 MiB, above the fixed 4 MiB
        a, b = _pair(13, 20, 512)
        ha, hb = ctx.mps_create(a), ctx.mps_create(b)
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(B.SmpsError) as e:
            ctx.scprod_noalloc(ha, hb, out.data_ptr())
        assert e.value.code == B.ENOMEM
        assert "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert float(out.item()) == 0.0
        ha.destroy()
        hb.destroy()
    finally:
        ctx.close()
