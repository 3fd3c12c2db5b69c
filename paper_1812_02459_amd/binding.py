"""ctypes binding of liblbm2p.so (include/lbm2p.h): argument marshalling only.

Every compute step runs in the HIP library; torch supplies device memory and the
stream.  Importing this module without the built library raises immediately:
there is no fallback path.
"""

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime under the same soname as the system one
# (libamdhip64.so.7); whichever is loaded first serves the whole process.  Load
# torch's before the library so that torch and the library share one runtime
# (the library is handed torch's memory and streams).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm2p.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOSPACE, EHIP, ENONFINITE, ESTATE = range(6)
OPT_STRAIN_MOMENTS, OPT_GI_LITERAL = 1, 2
PASSES = {"gather": 0, "fd": 1, "vel": 2, "filter": 3, "collide": 4}
FIELDS = {"phibar": 0, "praw": 1, "jx": 2, "jy": 3, "uKx": 4, "uKy": 5, "phi1": 6, "phi2": 7}


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("wall_x", ctypes.c_int32), ("wall_y", ctypes.c_int32),
        ("coupled", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
        ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("lam", ctypes.c_double), ("tau_f", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("filter_n", ctypes.c_int32), ("compact", ctypes.c_int32),
        ("compact_n", ctypes.c_int32), ("K", ctypes.c_int32),
        ("filter_a", ctypes.c_double), ("compact_alpha", ctypes.c_double),
        ("s_f", ctypes.c_double * 9), ("s_g", ctypes.c_double * 9),
        ("eps", ctypes.c_double),
        ("original_ch", ctypes.c_int32), ("options", ctypes.c_int32),
        ("p_ref", ctypes.c_double),
    ]


class AdjointIO(ctypes.Structure):
    _fields_ = [
        ("dL_dphi", ctypes.c_void_p), ("dL_df", ctypes.c_void_p), ("dL_dg", ctypes.c_void_p),
        ("dL_du", ctypes.c_void_p), ("phi0", ctypes.c_void_p), ("ux0", ctypes.c_void_p),
        ("uy0", ctypes.c_void_p), ("dL_dphi0", ctypes.c_void_p), ("dL_df0", ctypes.c_void_p),
        ("dL_dg0", ctypes.c_void_p), ("dL_du0", ctypes.c_void_p),
        ("dL_dsigma", ctypes.c_double), ("dL_dM", ctypes.c_double),
    ]


class LBMError(RuntimeError):
    pass


_vp = ctypes.c_void_p
_sig = {
    "lbm2p_workspace_bytes": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
    "lbm2p_create": [ctypes.POINTER(Params), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
    "lbm2p_init_fields": [_vp, _vp, _vp, _vp, _vp],
    "lbm2p_step": [_vp, ctypes.c_int32],
    "lbm2p_moments": [_vp, _vp, _vp, _vp, _vp, _vp],
    "lbm2p_fields": [_vp, ctypes.c_int32, _vp],
    "lbm2p_volume": [_vp, ctypes.POINTER(ctypes.c_double)],
    "lbm2p_get_state": [_vp, _vp, _vp, _vp],
    "lbm2p_set_state": [_vp, _vp, _vp, _vp],
    "lbm2p_profile": [_vp, ctypes.c_int32],
    "lbm2p_profile_read": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "lbm2p_adjoint_workspace_bytes": [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_size_t)],
    "lbm2p_record": [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t],
    "lbm2p_adjoint": [_vp, ctypes.POINTER(AdjointIO)],
    "lbm2p_stream_copy": [_vp, _vp, ctypes.c_size_t, _vp],
    "lbm2p_bubble": [_vp, ctypes.POINTER(ctypes.c_double)],
    "lbm2p_pressure_jump": [_vp, ctypes.POINTER(ctypes.c_double)],
    "lbm2p_track_residual": [_vp, ctypes.c_int32],
    "lbm2p_residual": [_vp, ctypes.POINTER(ctypes.c_double)],
    "lbm2p_set_velocity": [_vp, _vp, _vp],
    "lbm2p_volume_noalloc": [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.lbm2p_destroy.argtypes = [_vp]
_lib.lbm2p_destroy.restype = None
_lib.lbm2p_strerror.argtypes = [ctypes.c_int]
_lib.lbm2p_strerror.restype = ctypes.c_char_p

EXPORTED = list(_sig) + ["lbm2p_destroy", "lbm2p_strerror"]


def strerror(code):
    return _lib.lbm2p_strerror(code).decode()


def _check(code, what):
    if code != OK:
        raise LBMError(f"{what}: {strerror(code)} ({code})")
    return code


def make_params(d, precision=0):
    """lbm2p_params from a parameter dict (paper_1812_02459_amd.inputs.base_params keys)."""
    p = Params()
    p.nx, p.ny = int(d["nx"]), int(d["ny"])
    p.wall_x, p.wall_y = int(bool(d["wall_x"])), int(bool(d["wall_y"]))
    p.coupled = int(bool(d["coupled"]))
    p.precision = int(precision)
    for k in ("rho1", "rho2", "mu1", "mu2", "sigma", "W", "M", "lam", "tau_f", "gx", "gy",
              "rho_ref", "filter_a", "compact_alpha", "eps"):
        setattr(p, k, float(d[k]))
    p.filter_n = int(d["filter_n"])
    p.compact = int(bool(d["compact"]))
    p.compact_n = int(d["compact_n"])
    p.K = int(d["K"])
    sf = d.get("s_f", (1.0, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, 1.0, 1.0))
    sg = d.get("s_g", (1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.0, 0.0))
    for k in range(9):
        p.s_f[k] = 0.0 if sf[k] is None else float(sf[k])
        p.s_g[k] = 0.0 if sg[k] is None else float(sg[k])
    p.original_ch = int(bool(d.get("original_ch", False)))
    p.options = (OPT_STRAIN_MOMENTS if d.get("strain_moments", False) else 0) | \
        (OPT_GI_LITERAL if d.get("gi_literal", False) else 0)
    p.p_ref = float(d.get("p_ref", 0.0))
    return p


# ------------------------------------------------------------ raw C-ABI calls
def lbm2p_workspace_bytes(p):
    n = ctypes.c_size_t(0)
    _check(_lib.lbm2p_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "lbm2p_workspace_bytes")
    return n.value


def lbm2p_create(p, ws_ptr, nbytes, stream_ptr):
    out = _vp()
    _check(_lib.lbm2p_create(ctypes.byref(p), _vp(ws_ptr), nbytes, _vp(stream_ptr),
                             ctypes.byref(out)), "lbm2p_create")
    return out


def lbm2p_init_fields(ctx, phi0, ux0, uy0, p0):
    _check(_lib.lbm2p_init_fields(ctx, _vp(phi0), _vp(ux0), _vp(uy0), _vp(p0)),
           "lbm2p_init_fields")


def lbm2p_set_velocity(ctx, ux, uy):
    _check(_lib.lbm2p_set_velocity(ctx, _vp(ux), _vp(uy)), "lbm2p_set_velocity")


def lbm2p_step(ctx, n):
    _check(_lib.lbm2p_step(ctx, int(n)), "lbm2p_step")


def lbm2p_moments(ctx, phi, ux, uy, p, rho):
    _check(_lib.lbm2p_moments(ctx, _vp(phi), _vp(ux), _vp(uy), _vp(p), _vp(rho)),
           "lbm2p_moments")


def lbm2p_fields(ctx, which, out):
    _check(_lib.lbm2p_fields(ctx, int(which), _vp(out)), "lbm2p_fields")


def lbm2p_volume(ctx):
    out = (ctypes.c_double * 6)()
    code = _lib.lbm2p_volume(ctx, out)
    if code not in (OK, ENONFINITE):
        _check(code, "lbm2p_volume")
    return code, list(out)


def lbm2p_volume_noalloc(phi, p, ux, uy, nx, ny, out, stream_ptr):
    _check(_lib.lbm2p_volume_noalloc(_vp(phi), _vp(p), _vp(ux), _vp(uy), int(nx), int(ny),
                                     _vp(out), _vp(stream_ptr)), "lbm2p_volume_noalloc")


def lbm2p_bubble(ctx):
    out = (ctypes.c_double * 3)()
    _check(_lib.lbm2p_bubble(ctx, out), "lbm2p_bubble")
    return list(out)


def lbm2p_track_residual(ctx, on):
    _check(_lib.lbm2p_track_residual(ctx, int(on)), "lbm2p_track_residual")


def lbm2p_residual(ctx):
    out = ctypes.c_double()
    _check(_lib.lbm2p_residual(ctx, ctypes.byref(out)), "lbm2p_residual")
    return out.value


def lbm2p_pressure_jump(ctx):
    out = (ctypes.c_double * 5)()
    _check(_lib.lbm2p_pressure_jump(ctx, out), "lbm2p_pressure_jump")
    return list(out)


def lbm2p_get_state(ctx, f, g, u):
    _check(_lib.lbm2p_get_state(ctx, _vp(f), _vp(g), _vp(u)), "lbm2p_get_state")


def lbm2p_set_state(ctx, f, g, u):
    _check(_lib.lbm2p_set_state(ctx, _vp(f), _vp(g), _vp(u)), "lbm2p_set_state")


def lbm2p_profile(ctx, pass_id):
    _check(_lib.lbm2p_profile(ctx, int(pass_id)), "lbm2p_profile")


def lbm2p_profile_read(ctx):
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(_lib.lbm2p_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n)), "lbm2p_profile_read")
    return ms.value, n.value


def lbm2p_adjoint_workspace_bytes(p, nsteps, ckpt_every):
    n = ctypes.c_size_t(0)
    _check(_lib.lbm2p_adjoint_workspace_bytes(ctypes.byref(p), int(nsteps), int(ckpt_every),
                                              ctypes.byref(n)), "lbm2p_adjoint_workspace_bytes")
    return n.value


def lbm2p_record(ctx, nsteps, ckpt_every, ws_ptr, nbytes):
    _check(_lib.lbm2p_record(ctx, int(nsteps), int(ckpt_every), _vp(ws_ptr), nbytes),
           "lbm2p_record")


def lbm2p_adjoint(ctx, io):
    _check(_lib.lbm2p_adjoint(ctx, ctypes.byref(io)), "lbm2p_adjoint")
    return io.dL_dsigma, io.dL_dM


def lbm2p_stream_copy(src_ptr, dst_ptr, nbytes, stream_ptr):
    _check(_lib.lbm2p_stream_copy(_vp(src_ptr), _vp(dst_ptr), int(nbytes), _vp(stream_ptr)),
           "lbm2p_stream_copy")


def lbm2p_destroy(ctx):
    _lib.lbm2p_destroy(ctx)


# ------------------------------------------------------------------ wrapper
class Sim:
    """A context with a torch-owned workspace on the current device and stream."""

    def __init__(self, params, precision=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.coupled = bool(params["coupled"])
        self.device = torch.device(device)
        self.p = make_params(params, precision)
        nbytes = lbm2p_workspace_bytes(self.p)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = lbm2p_create(self.p, aligned, nbytes, self.stream.cuda_stream)

    def _dev(self, a):
        t = self.torch
        if a is None:
            return None
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        return a.to(device=self.device, dtype=t.float64).contiguous()

    def init(self, phi0, ux0=None, uy0=None, p0=None):
        self._keep = [self._dev(a) for a in (phi0, ux0, uy0, p0)]
        ptr = [a.data_ptr() if a is not None else None for a in self._keep]
        lbm2p_init_fields(self.ctx, *ptr)
        return self

    def step(self, n=1):
        lbm2p_step(self.ctx, n)
        return self

    def set_velocity(self, ux, uy):
        """CH-only mode: the prescribed velocity of the following steps."""
        ux, uy = self._dev(ux), self._dev(uy)
        lbm2p_set_velocity(self.ctx, ux.data_ptr(), uy.data_ptr())
        self._vel = (ux, uy)          # alive until the stream has consumed them
        return self

    def _plane(self):
        return self.torch.empty((self.ny, self.nx), dtype=self.torch.float64, device=self.device)

    def moments(self):
        phi, ux, uy, p, rho = (self._plane() for _ in range(5))
        lbm2p_moments(self.ctx, phi.data_ptr(), ux.data_ptr(), uy.data_ptr(), p.data_ptr(),
                      rho.data_ptr())
        return dict(phi=phi, ux=ux, uy=uy, p=p, rho=rho)

    def field(self, name):
        out = self._plane()
        lbm2p_fields(self.ctx, FIELDS[name], out.data_ptr())
        return out

    def volume(self):
        code, v = lbm2p_volume(self.ctx)
        return dict(count=v[0], sum_phi=v[1], sum_p=v[2], max_u=v[3], min_phi=v[4],
                    max_phi=v[5], finite=(code == OK))

    def bubble(self):
        """Area (node count), y_c and V_c of the region phi < 0 (eq:quantify-yc,
        eq:quantify-uc); y in row indices."""
        a, yc, vc = lbm2p_bubble(self.ctx)
        return dict(area=a, y_c=yc, V_c=vc)

    def track_residual(self, on=True):
        """Keep the velocity iteration's residual of the following steps."""
        lbm2p_track_residual(self.ctx, 1 if on else 0)

    def residual(self):
        """zeta = sum |u^K - u^{K-1}| / sum |u^{K-1}| of the last (tracked) step."""
        return lbm2p_residual(self.ctx)

    def pressure_jump(self):
        """<rho p~> over phi > 0.99 minus over phi < -0.99 (Sec. 4.3), the two means
        and the two node counts."""
        d, pin, pout, nin, nout = lbm2p_pressure_jump(self.ctx)
        return dict(dp=d, p_in=pin, p_out=pout, n_in=nin, n_out=nout)

    def get_state(self):
        t = self.torch
        f = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
        g = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device) \
            if self.coupled else None
        u = t.empty((2, self.ny, self.nx), dtype=t.float64, device=self.device)
        lbm2p_get_state(self.ctx, f.data_ptr(), g.data_ptr() if g is not None else None,
                        u.data_ptr())
        return f, g, u

    def set_state(self, f, g, u):
        f, g, u = self._dev(f), self._dev(g), self._dev(u)
        lbm2p_set_state(self.ctx, f.data_ptr(), g.data_ptr() if g is not None else None,
                        u.data_ptr())
        self.torch.cuda.current_stream(self.device).synchronize()
        return self

    def record(self, nsteps, ckpt_every=64):
        """Advance nsteps steps keeping the checkpoints the adjoint needs."""
        nbytes = lbm2p_adjoint_workspace_bytes(self.p, nsteps, ckpt_every)
        self.adj_ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        aligned = (self.adj_ws.data_ptr() + 255) // 256 * 256
        lbm2p_record(self.ctx, nsteps, ckpt_every, aligned, nbytes)
        return self

    def adjoint(self, dL_dphi=None, dL_df=None, dL_dg=None, dL_du=None, want_phi0=False,
                want_state=False):
        """Reverse mode of the last record(): seeds on the final phi / state,
        returns dL/dsigma, dL/dM and (on request) dL/dphi0 and the adjoint of
        the recorded run's initial state."""
        t = self.torch
        seeds = [self._dev(a) for a in (dL_dphi, dL_df, dL_dg, dL_du)]
        io = AdjointIO()
        for name, a in zip(("dL_dphi", "dL_df", "dL_dg", "dL_du"), seeds):
            setattr(io, name, a.data_ptr() if a is not None else None)
        out = {}
        if want_phi0:
            phi0, ux0, uy0 = self._keep[0], self._keep[1], self._keep[2]
            io.phi0 = phi0.data_ptr()
            io.ux0 = ux0.data_ptr() if ux0 is not None else None
            io.uy0 = uy0.data_ptr() if uy0 is not None else None
            out["phi0"] = self._plane()
            io.dL_dphi0 = out["phi0"].data_ptr()
        if want_state:
            out["f0"] = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
            io.dL_df0 = out["f0"].data_ptr()
            if self.coupled:
                out["g0"] = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
                io.dL_dg0 = out["g0"].data_ptr()
            out["u0"] = t.empty((2, self.ny, self.nx), dtype=t.float64, device=self.device)
            io.dL_du0 = out["u0"].data_ptr()
        out["sigma"], out["M"] = lbm2p_adjoint(self.ctx, io)
        return out

    def profile(self, pass_name):
        lbm2p_profile(self.ctx, -1 if pass_name is None else PASSES[pass_name])

    def profile_read(self):
        return lbm2p_profile_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbm2p_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class PhaseFieldRun(torch.autograd.Function):
        """(sigma, M, phi0) -> phi after nsteps steps, with the HIP adjoint as
        its backward (checkpoints every ckpt_every steps).  sigma and M are
        0-dim float64 tensors, phi0 a (ny, nx) float64 tensor; params holds
        every other parameter; ux0, uy0, p0 are constants."""

        @staticmethod
        def forward(ctx, sigma, M, phi0, params, nsteps, ckpt_every=64, precision=0, ux0=None,
                    uy0=None, p0=None):
            prm = dict(params)
            prm["sigma"] = float(sigma)
            prm["M"] = float(M)
            dev = phi0.device if phi0.is_cuda else torch.device("cuda:0")
            sim = Sim(prm, precision=precision, device=dev)
            sim.init(phi0.detach(), ux0, uy0, p0)
            sim.record(nsteps, ckpt_every)
            ctx.sim = sim
            return sim.moments()["phi"].to(phi0.device)

        @staticmethod
        def backward(ctx, g):
            sim = ctx.sim
            out = sim.adjoint(dL_dphi=g, want_phi0=True)
            ctx.sim = None
            sim.close()
            dt = torch.float64
            return (torch.tensor(out["sigma"], dtype=dt), torch.tensor(out["M"], dtype=dt),
                    out["phi0"].to(g.device), None, None, None, None, None, None, None)

    return PhaseFieldRun


def phase_field_run(sigma, M, phi0, params, nsteps, ckpt_every=64, precision=0, ux0=None,
                    uy0=None, p0=None):
    """Differentiable run: phi_T as a function of (sigma, M, phi0)."""
    global _PFR
    if _PFR is None:
        _PFR = _autograd_function()
    return _PFR.apply(sigma, M, phi0, params, nsteps, ckpt_every, precision, ux0, uy0, p0)


_PFR = None
