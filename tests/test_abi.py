"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/lbm2p.h declares, sizes workspaces and rejects invalid
parameters with the documented error codes."""

import ctypes
import os
import re

import pytest

from paper_1812_02459_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm2p.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm2p_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1812_02459_amd import binding as B
    names = _declared()
    assert len(names) >= 13
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_workspace_and_validation():
    from paper_1812_02459_amd import binding as B
    ok = I.base_params(64, 48)
    n64 = B.lbm2p_workspace_bytes(B.make_params(ok, 0))
    n32 = B.lbm2p_workspace_bytes(B.make_params(ok, 1))
    assert n64 > 34 * 64 * 48 * 8 and n32 < n64
    nc = B.lbm2p_workspace_bytes(B.make_params(dict(ok, compact=True), 0))
    assert nc > n64                                        # line scratch and tables
    ch = dict(ok, coupled=False)
    assert B.lbm2p_workspace_bytes(B.make_params(ch, 0)) < n64
    bad = [dict(ok, nx=15), dict(ok, rho2=0.0), dict(ok, tau_f=0.5), dict(ok, filter_n=6),
           dict(ok, K=0), dict(ok, K=9), dict(ok, filter_a=1.5), dict(ok, W=0.0),
           dict(ok, eps=-1.0), dict(ok, mu1=-1.0), dict(ok, compact=True, compact_n=6),
           dict(ok, compact=True, compact_alpha=0.5), dict(ok, compact=True, compact_n=0),
           dict(ok, compact=True, nx=7681), dict(ok, p_ref=float("nan")),
           dict(ok, p_ref=float("inf")), dict(ok, coupled=False, strain_moments=True),
           dict(ok, coupled=False, gi_literal=True)]
    for b in bad:
        with pytest.raises(B.LBMError, match="invalid argument"):
            B.lbm2p_workspace_bytes(B.make_params(b, 0))
    p = B.make_params(ok, 0)
    p.s_g[1] = 2.5
    with pytest.raises(B.LBMError):
        B.lbm2p_workspace_bytes(p)


def test_create_checks_workspace_without_touching_the_device():
    from paper_1812_02459_amd import binding as B
    p = B.make_params(I.base_params(32, 32), 0)
    need = B.lbm2p_workspace_bytes(p)
    buf = ctypes.create_string_buffer(512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    with pytest.raises(B.LBMError, match="workspace too small"):
        B.lbm2p_create(p, aligned, need - 1, None)
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_create(p, aligned + 8, need, None)          # misaligned
    ctx = B.lbm2p_create(p, aligned, need, None)           # host-side only
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_step(ctx, 1)                               # before init
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_step(ctx, -1)
    B.lbm2p_destroy(ctx)
    assert B.strerror(4) == "non-finite value in the state"


def test_adjoint_workspace_and_state_checks_without_touching_the_device():
    from paper_1812_02459_amd import binding as B
    ok = I.base_params(64, 48)
    p = B.make_params(ok, 0)
    n0 = B.lbm2p_adjoint_workspace_bytes(p, 0, 64)
    n1 = B.lbm2p_adjoint_workspace_bytes(p, 640, 64)
    n2 = B.lbm2p_adjoint_workspace_bytes(p, 640, 8)
    n3 = B.lbm2p_adjoint_workspace_bytes(p, 640, 32)
    # checkpoints (22 planes each) every k steps against k per-step slots (12 planes
    # each): the total is smallest near k = sqrt(640 * 22 / 12) ~ 34
    assert 0 < n0 < n1 and n3 < n1 and n3 < n2
    assert B.lbm2p_adjoint_workspace_bytes(B.make_params(ok, 1), 640, 64) < n1
    for bad in [dict(nsteps=-1, k=4), dict(nsteps=10, k=0)]:
        with pytest.raises(B.LBMError, match="invalid argument"):
            B.lbm2p_adjoint_workspace_bytes(p, bad["nsteps"], bad["k"])
    # the compact filter has an adjoint too; its workspace matches the explicit filter's
    nca = B.lbm2p_adjoint_workspace_bytes(B.make_params(dict(ok, compact=True), 0), 10, 4)
    assert nca == B.lbm2p_adjoint_workspace_bytes(B.make_params(ok, 0), 10, 4)
    need = B.lbm2p_workspace_bytes(p)
    buf = ctypes.create_string_buffer(need + 512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    ctx = B.lbm2p_create(p, aligned, need, None)           # host-side only
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_record(ctx, 4, 2, aligned, need)           # before init
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_record(ctx, 4, 0, aligned, need)
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_adjoint(ctx, B.AdjointIO())                # nothing recorded
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_bubble(ctx)                                # before init
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_pressure_jump(ctx)                         # before init
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_track_residual(ctx, 2)
    B.lbm2p_track_residual(ctx, 1)                         # host-side switch
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_residual(ctx)                              # no tracked step yet
    B.lbm2p_destroy(ctx)
    ch = B.make_params(dict(ok, coupled=False), 0)
    need = B.lbm2p_workspace_bytes(ch)
    buf = ctypes.create_string_buffer(need + 512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    ctx = B.lbm2p_create(ch, aligned, need, None)
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_pressure_jump(ctx)                         # no pressure in CH-only mode
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_residual(ctx)                              # no velocity iteration either
    with pytest.raises(B.LBMError, match="call out of order"):
        B.lbm2p_set_velocity(ctx, base := 1 << 20, base)   # before init
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_set_velocity(ctx, None, 1 << 20)
    B.lbm2p_destroy(ctx)
    cp = B.make_params(ok, 0)
    need = B.lbm2p_workspace_bytes(cp)
    buf = ctypes.create_string_buffer(need + 512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    ctx = B.lbm2p_create(cp, aligned, need, None)
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_set_velocity(ctx, 1 << 20, 1 << 20)        # coupled: u solves Eq:u
    B.lbm2p_destroy(ctx)
    # options: unknown bits are invalid; the adjoint covers the default readings only
    bad = B.make_params(ok, 0)
    bad.options = 4
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_workspace_bytes(bad)
    op = B.make_params(dict(ok, strain_moments=True), 0)
    assert op.options == B.OPT_STRAIN_MOMENTS
    need_o = B.lbm2p_workspace_bytes(op)
    assert need_o > need                                   # m_1, m_7, m_8 planes
    buf = ctypes.create_string_buffer(need_o + 512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    ctx = B.lbm2p_create(op, aligned, need_o, None)
    with pytest.raises(B.LBMError, match="invalid argument"):
        B.lbm2p_record(ctx, 4, 2, aligned, need_o)
    B.lbm2p_destroy(ctx)


def test_stream_copy_argument_checks_without_touching_the_device():
    from paper_1812_02459_amd import binding as B
    B.lbm2p_stream_copy(None, None, 0, None)                # nothing to copy
    base = 1 << 20
    for src, dst, n in [(None, base, 16), (base, None, 16), (base + 8, base + 4096, 16),
                        (base, base + 4100, 16), (base, base + 32, 64), (base + 32, base, 64)]:
        with pytest.raises(B.LBMError, match="invalid argument"):
            B.lbm2p_stream_copy(src, dst, n, None)
