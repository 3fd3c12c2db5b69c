"""lbm2p_volume_noalloc, the diagnostics entry point that allocates nothing
(its partials live in the library's static device array), against
lbm2p_volume on the same state: two calls in a row, the second on a smaller
lattice, then a CH-only state without a pressure plane.  From an FP64 context
the values are bitwise equal (the same reduction in the same order); from an
FP32 context the count and the extrema are equal and the float64 sums agree to
1e-15 (the FP32 unit may contract the |u| products into fused multiply-adds)."""

import pytest
import torch

from paper_1812_02459_amd import inputs as I

from gpu_common import gpu_sim, droplet_case

pytestmark = pytest.mark.gpu


def _noalloc(sim, with_p=True):
    from paper_1812_02459_amd import binding as B
    m = sim.moments()
    out = torch.full((6,), float("nan"), dtype=torch.float64, device=sim.device)
    p = m["p"].data_ptr() if with_p else None
    B.lbm2p_volume_noalloc(m["phi"].data_ptr(), p, m["ux"].data_ptr(), m["uy"].data_ptr(),
                           sim.nx, sim.ny, out.data_ptr(), sim.stream.cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().tolist()


def _compare(sim, got, exact):
    from paper_1812_02459_amd.binding import lbm2p_volume, OK
    code, ref = lbm2p_volume(sim.ctx)
    print(sim.nx, sim.ny, "volume", ref, "noalloc", got, flush=True)
    assert code == OK
    if exact:
        assert got == ref
    else:
        assert got[0] == ref[0] and got[4] == ref[4] and got[5] == ref[5]
        for k in (1, 2, 3):
            assert abs(got[k] - ref[k]) <= 1e-15 * max(abs(ref[k]), 1e-300) * 10
    assert ref[0] > 0


def test_volume_noalloc_matches_volume_on_consecutive_calls():
    big = gpu_sim(droplet_case(200, 180, seed=31))
    big.step(3)
    _compare(big, _noalloc(big), exact=True)
    small = gpu_sim(droplet_case(48, 40, seed=32, wall_y=True))
    small.step(2)
    _compare(small, _noalloc(small), exact=True)
    vort = gpu_sim(I.vortex(n=64))
    vort.step(5)
    _compare(vort, _noalloc(vort, with_p=False), exact=True)
    for s in (big, small, vort):
        s.close()


def test_volume_noalloc_from_fp32_contexts():
    a = gpu_sim(droplet_case(96, 80, seed=33), precision=1)
    a.step(4)
    _compare(a, _noalloc(a), exact=False)
    b = gpu_sim(droplet_case(40, 32, seed=34), precision=1)
    b.step(1)
    _compare(b, _noalloc(b), exact=False)
    a.close()
    b.close()


def test_volume_noalloc_rejects_invalid_arguments():
    from paper_1812_02459_amd import binding as B
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    ptr = x.data_ptr()
    for args in [(None, None, ptr, ptr, 2, 2, ptr), (ptr, None, ptr, ptr, 0, 2, ptr),
                 (ptr, None, ptr, ptr, 2, 2, None), (ptr, None, ptr, ptr, 1 << 16, 1 << 16, ptr)]:
        with pytest.raises(B.LBMError, match="invalid argument"):
            B.lbm2p_volume_noalloc(*args, None)
