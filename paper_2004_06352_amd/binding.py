"""Python binding of the C ABI in ``include/lenshpc.h`` (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch provides device memory and the current stream.  The library
must have been built (``python -m paper_2004_06352_amd.build``); nothing here
falls back to any other implementation.

Containers
  table    dict of float64 device tensors x0, y0, b0, eps, phi, rcore, rcut
  phys     dict of float64 device tensors x0, y0, sigma, e, phi, rcore, rcut
  grid     (nx, ny, x0, y0, dx, dy)
  catalog  dict: off (int32), x, y, sig (float64 per image), f (float64 Dls/Ds per system)
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # load torch's HIP runtime before the library (one runtime per process)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_native", "liblenshpc.so")

FP64, FP32_ACC64, FP32_COMP32 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32_acc64": FP32_ACC64, "fp32_comp32": FP32_COMP32}
CHI2_SOURCE, CHI2_IMAGE = 0, 1
PATH_BATCHED, PATH_PER_SAMPLE = 0, 1
CTX_CHECK_TABLES = 1

STATUS = {0: "LENS_OK", -1: "LENS_EINVAL", -2: "LENS_ENOMEM", -3: "LENS_EDEVICE",
          -4: "LENS_EOVERFLOW", -5: "LENS_EUNSUPPORTED"}

POT_KEYS = ("x0", "y0", "b0", "eps", "phi", "rcore", "rcut")
PHYS_KEYS = ("x0", "y0", "sigma", "e", "phi", "rcore", "rcut")

EXPORTS = ("lens_ctx_create", "lens_ctx_destroy", "lens_ctx_status", "lens_set_map_tuning",
           "lens_get_map_tuning", "lens_set_chi2_tuning", "lens_get_chi2_tuning",
           "lens_table_from_physical", "lens_grad_map",
           "lens_hessian_map", "lens_hessian_map_noalloc", "lens_derived_map", "lens_potential_map", "lens_time_delay_map",
           "lens_time_delay_scale", "lens_chi2_batch", "lens_find_images",
           "lens_chi2_plan_create", "lens_chi2_plan_create_ex", "lens_chi2_plan_create2",
           "lens_chi2_plan_launch", "lens_chi2_plan_status", "lens_chi2_plan_destroy", "lens_mcmc_create",
           "lens_mcmc_step", "lens_mcmc_destroy", "lens_dlsds",
           "lens_b0_from_sigma", "lens_eps_from_e", "lens_map_scratch_bytes",
           "lens_chi2_scratch_bytes", "lens_last_error", "lens_abi_version")


class LensError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Pot(C.Structure):
    _fields_ = [("n", C.c_int32)] + [(k, C.c_void_p) for k in POT_KEYS]


class _Phys(C.Structure):
    _fields_ = [("n", C.c_int32)] + [(k, C.c_void_p) for k in PHYS_KEYS]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("y0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double)]


class _Batch(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("free_offset", C.c_void_p), ("free", _Pot),
                ("fixed", _Pot)]


class _Cat(C.Structure):
    _fields_ = [("n_sys", C.c_int32), ("n_img", C.c_int32), ("img_offset", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("sigma", C.c_void_p),
                ("dlsds", C.c_void_p)]


class _McmcDesc(C.Structure):
    _fields_ = [("n_walkers", C.c_int32), ("n_free", C.c_int32), ("params", C.c_void_p),
                ("chi2", C.c_void_p), ("accepted", C.c_void_p), ("lo", C.c_void_p),
                ("hi", C.c_void_p), ("step", C.c_void_p), ("u", C.c_void_p),
                ("convention", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("prec", C.c_int32), ("path", C.c_int32), ("grid", _Grid),
                ("max_img_per_sys", C.c_int32), ("missing_penalty", C.c_double),
                ("refine_max_iter", C.c_int32), ("refine_tol", C.c_double)]


class MapTuning(C.Structure):
    _fields_ = [("block_x", C.c_int32), ("block_y", C.c_int32), ("pix_per_thread", C.c_int32),
                ("stage", C.c_int32), ("lds_chunk", C.c_int32)]

    def as_tuple(self):
        return (self.block_x, self.block_y, self.pix_per_thread, self.stage, self.lds_chunk)


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(python -m paper_2004_06352_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.lens_ctx_create.argtypes = [i32, C.c_uint64, C.c_uint32, C.POINTER(vp)]
        L.lens_ctx_destroy.argtypes = [vp]
        L.lens_ctx_status.argtypes = [vp]
        L.lens_set_map_tuning.argtypes = [vp, i32, C.POINTER(MapTuning)]
        L.lens_get_map_tuning.argtypes = [vp, i32, C.POINTER(MapTuning)]
        L.lens_set_chi2_tuning.argtypes = [vp, i32]
        L.lens_get_chi2_tuning.argtypes = [vp, C.POINTER(i32)]
        L.lens_table_from_physical.argtypes = [vp, C.POINTER(_Phys), i32, vp, vp, vp]
        L.lens_grad_map.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, i32, vp, vp, vp]
        L.lens_hessian_map.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, i32, vp, vp,
                                       vp, vp, vp, vp]
        L.lens_hessian_map_noalloc.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, i32,
                                               vp, vp, vp, vp, vp, vp]
        L.lens_derived_map.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, i32, vp, vp,
                                       vp, vp, vp, vp, vp]
        L.lens_potential_map.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, i32, vp, vp]
        L.lens_time_delay_map.argtypes = [vp, C.POINTER(_Pot), C.POINTER(_Grid), dbl, dbl, dbl,
                                          dbl, vp, vp]
        L.lens_time_delay_scale.argtypes = [dbl, dbl, dbl, dbl, dbl, C.POINTER(dbl)]
        L.lens_chi2_batch.argtypes = [vp, C.POINTER(_Batch), C.POINTER(_Cat), C.POINTER(_Opts),
                                      vp, vp, vp, vp, vp]
        L.lens_find_images.argtypes = [vp, vp, vp, C.POINTER(_Grid), i32, vp, vp, vp, i32, vp,
                                       vp, vp, vp, vp]
        L.lens_chi2_plan_create.argtypes = [vp, C.POINTER(_Batch), C.POINTER(_Cat),
                                            C.POINTER(_Opts), vp, vp, C.POINTER(vp)]
        L.lens_chi2_plan_create_ex.argtypes = [vp, C.POINTER(_Batch), C.POINTER(_Cat),
                                               C.POINTER(_Opts), vp, C.c_uint32, vp,
                                               C.POINTER(vp)]
        L.lens_chi2_plan_create2.argtypes = [vp, C.POINTER(_Batch), C.POINTER(_Cat),
                                             C.POINTER(_Opts), vp, vp, vp, vp, C.c_uint32, vp,
                                             C.POINTER(vp)]
        L.lens_chi2_plan_launch.argtypes = [vp, vp]
        L.lens_chi2_plan_status.argtypes = [vp, vp]
        L.lens_chi2_plan_destroy.argtypes = [vp]
        L.lens_dlsds.argtypes = [dbl, dbl, dbl, dbl, C.POINTER(dbl)]
        L.lens_b0_from_sigma.argtypes = [dbl, i32, C.POINTER(dbl)]
        L.lens_eps_from_e.argtypes = [dbl, C.POINTER(dbl)]
        L.lens_map_scratch_bytes.argtypes = [i32, C.POINTER(C.c_uint64)]
        L.lens_chi2_scratch_bytes.argtypes = [i32, i32, i32, i32, i32, C.POINTER(_Opts),
                                              C.POINTER(C.c_uint64)]
        L.lens_last_error.restype = C.c_char_p
        L.lens_abi_version.restype = i32
        for name in EXPORTS:
            if name not in ("lens_last_error", "lens_abi_version"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise LensError(status, lib().lens_last_error().decode())


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """A library context on one device (scratch + flags).  check=True
    validates table contents before each launch (synchronising once)."""

    def __init__(self, device: int = 0, scratch_max: int = 16 << 30, check: bool = True):
        self.device = device
        h = C.c_void_p()
        _check(lib().lens_ctx_create(device, scratch_max, CTX_CHECK_TABLES if check else 0,
                                     C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().lens_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def status(self):
        _check(lib().lens_ctx_status(self.handle))

    def set_map_tuning(self, prec, tuning=None):
        if tuning is not None and not isinstance(tuning, MapTuning):
            tuning = MapTuning(*tuning)
        _check(lib().lens_set_map_tuning(self.handle, prec,
                                         C.byref(tuning) if tuning is not None else None))

    def get_map_tuning(self, prec):
        t = MapTuning()
        _check(lib().lens_get_map_tuning(self.handle, prec, C.byref(t)))
        return t.as_tuple()

    def set_chi2_tuning(self, waves_per_cu):
        _check(lib().lens_set_chi2_tuning(self.handle, int(waves_per_cu)))

    def get_chi2_tuning(self):
        v = C.c_int32()
        _check(lib().lens_get_chi2_tuning(self.handle, C.byref(v)))
        return v.value


_contexts = {}


def default_context(device=None, check=True) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    key = (device, check)
    if key not in _contexts:
        _contexts[key] = Context(device, check=check)
    return _contexts[key]


def _dev(t, device, dtype=torch.float64):
    t = torch.as_tensor(t, dtype=dtype)
    return t.to(device=device).contiguous()


def to_device(d: dict, keys, device="cuda"):
    """dict of array-likes -> dict of contiguous float64 device tensors."""
    return {k: _dev(d[k], device) for k in keys}


def _pot(t):
    n = int(t["x0"].numel())
    for k in POT_KEYS:
        assert t[k].dtype == torch.float64 and t[k].is_cuda and t[k].is_contiguous(), k
        assert t[k].numel() == n, k
    return _Pot(n, *[t[k].data_ptr() if n else None for k in POT_KEYS])


def _grid(g):
    nx, ny, x0, y0, dx, dy = g
    return _Grid(int(nx), int(ny), float(x0), float(y0), float(dx), float(dy))


def _ctx(ctx):
    return ctx if ctx is not None else default_context()


def table_from_physical(phys, convention=0, ctx=None):
    """Physical table -> amplitude table on the device (library prologue)."""
    ctx = _ctx(ctx)
    n = int(phys["x0"].numel())
    dev = phys["x0"].device
    b0 = torch.empty(n, dtype=torch.float64, device=dev)
    eps = torch.empty(n, dtype=torch.float64, device=dev)
    P = _Phys(n, *[phys[k].data_ptr() if n else None for k in PHYS_KEYS])
    _check(lib().lens_table_from_physical(ctx.handle, C.byref(P), convention,
                                          _ptr(b0) if n else None, _ptr(eps) if n else None,
                                          _stream(dev)))
    return dict(x0=phys["x0"], y0=phys["y0"], b0=b0, eps=eps, phi=phys["phi"],
                rcore=phys["rcore"], rcut=phys["rcut"])


def _out_dtype(prec):
    return torch.float64 if prec == FP64 else torch.float32


def grad_map(table, grid, dlsds=1.0, prec=FP64, ctx=None, out=None):
    """(ax, ay), each (ny, nx): dlsds times the summed deflection (into
    out["ax"], out["ay"] when given)."""
    ctx = _ctx(ctx)
    nx, ny = int(grid[0]), int(grid[1])
    dev = table["x0"].device
    if out is not None:
        ax, ay = out["ax"], out["ay"]
    else:
        ax = torch.empty((ny, nx), dtype=_out_dtype(prec), device=dev)
        ay = torch.empty_like(ax)
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_grad_map(ctx.handle, C.byref(T), C.byref(G), float(dlsds), prec,
                               _ptr(ax), _ptr(ay), _stream(dev)))
    return ax, ay


def hessian_map(table, grid, dlsds=1.0, prec=FP64, with_alpha=True, ctx=None, out=None):
    """dict of (ny, nx) planes hxx, hxy, hyy (and ax, ay when with_alpha)."""
    ctx = _ctx(ctx)
    nx, ny = int(grid[0]), int(grid[1])
    dev = table["x0"].device
    if out is None:
        names = ("hxx", "hxy", "hyy") + (("ax", "ay") if with_alpha else ())
        out = {k: torch.empty((ny, nx), dtype=_out_dtype(prec), device=dev) for k in names}
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_hessian_map(ctx.handle, C.byref(T), C.byref(G), float(dlsds), prec,
                                  _ptr(out["hxx"]), _ptr(out["hxy"]), _ptr(out["hyy"]),
                                  _ptr(out.get("ax")), _ptr(out.get("ay")), _stream(dev)))
    return out


# the allocation-free call's table limit (LENS_NOALLOC_MAX_POT)
NOALLOC_MAX_POT = 8192


def hessian_map_noalloc(table, grid, dlsds=1.0, prec=FP64, ctx=None, out=None):
    """lens_hessian_map_noalloc into the caller's planes `out` (dict hxx, hxy,
    hyy and optionally ax, ay); the library allocates nothing for the call."""
    ctx = _ctx(ctx)
    dev = table["x0"].device
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_hessian_map_noalloc(ctx.handle, C.byref(T), C.byref(G), float(dlsds),
                                          prec, _ptr(out["hxx"]), _ptr(out["hxy"]),
                                          _ptr(out["hyy"]), _ptr(out.get("ax")),
                                          _ptr(out.get("ay")), _stream(dev)))
    return out


DERIVED = ("kappa", "gamma1", "gamma2", "gamma", "mu", "det")


def derived_map(table, grid, dlsds=1.0, prec=FP64, names=DERIVED, ctx=None, out=None):
    """dict of (ny, nx) planes of the derived maps named in `names` (a subset
    of kappa, gamma1, gamma2, gamma, mu, det)."""
    ctx = _ctx(ctx)
    nx, ny = int(grid[0]), int(grid[1])
    dev = table["x0"].device
    if out is None:
        out = {k: torch.empty((ny, nx), dtype=_out_dtype(prec), device=dev) for k in names}
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_derived_map(ctx.handle, C.byref(T), C.byref(G), float(dlsds), prec,
                                  *[_ptr(out.get(k)) for k in DERIVED], _stream(dev)))
    return out


def potential_map(table, grid, dlsds=1.0, ctx=None, out=None):
    """(ny, nx) FP64 lensing potential."""
    ctx = _ctx(ctx)
    nx, ny = int(grid[0]), int(grid[1])
    dev = table["x0"].device
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float64, device=dev)
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_potential_map(ctx.handle, C.byref(T), C.byref(G), float(dlsds), FP64,
                                    _ptr(out), _stream(dev)))
    return out


def time_delay_map(table, grid, dlsds, beta, scale, ctx=None, out=None):
    """(ny, nx) FP64 time-delay surface scale (|theta - beta|^2 / 2 - psi)."""
    ctx = _ctx(ctx)
    nx, ny = int(grid[0]), int(grid[1])
    dev = table["x0"].device
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float64, device=dev)
    T, G = _pot(table), _grid(grid)
    _check(lib().lens_time_delay_map(ctx.handle, C.byref(T), C.byref(G), float(dlsds),
                                     float(beta[0]), float(beta[1]), float(scale), _ptr(out),
                                     _stream(dev)))
    return out


def time_delay_scale(zl, zs, h0=70.0, om=0.3, ol=0.7):
    """Days per arcsec^2 of the time-delay surface (host helper)."""
    v = C.c_double()
    _check(lib().lens_time_delay_scale(float(zl), float(zs), float(h0), float(om), float(ol),
                                       C.byref(v)))
    return v.value


def _batch(fixed, free, free_off):
    return _Batch(int(free_off.numel()) - 1, free_off.data_ptr(), _pot(free), _pot(fixed))


def _catalog(cat):
    off = cat["off"]
    assert off.dtype == torch.int32 and off.is_cuda
    return _Cat(int(off.numel()) - 1, int(cat["x"].numel()), off.data_ptr(), cat["x"].data_ptr(),
                cat["y"].data_ptr(), cat["sig"].data_ptr(), cat["f"].data_ptr())


def catalog_to_device(cat, device="cuda"):
    return dict(off=torch.as_tensor(cat["off"], dtype=torch.int32).to(device).contiguous(),
                x=_dev(cat["x"], device), y=_dev(cat["y"], device), sig=_dev(cat["sig"], device),
                f=_dev(cat["f"], device))


def _opts(mode, prec, path, grid, kmax, penalty, refine=None):
    g = _grid(grid) if grid is not None else _Grid(0, 0, 0, 0, 0, 0)
    it, tol = refine if refine is not None else (0, 0.0)
    return _Opts(mode, prec, path, g, int(kmax), float(penalty), int(it), float(tol))


def map_scratch_bytes(n_pot):
    """Context scratch of a map call over n_pot potentials (host arithmetic)."""
    out = C.c_uint64()
    _check(lib().lens_map_scratch_bytes(int(n_pot), C.byref(out)))
    return out.value


def chi2_scratch_bytes(n_fixed, n_free, n_samples, n_sys, n_img, mode=CHI2_SOURCE, prec=FP64,
                       path=PATH_BATCHED, grid=None, kmax=16):
    """Context scratch of a lens_chi2_batch call of these sizes (host arithmetic)."""
    o = _opts(mode, prec, path, grid, kmax, 0.0, None)
    out = C.c_uint64()
    _check(lib().lens_chi2_scratch_bytes(int(n_fixed), int(n_free), int(n_samples), int(n_sys),
                                         int(n_img), C.byref(o), C.byref(out)))
    return out.value


def chi2_batch(fixed, free, free_off, cat, mode=CHI2_SOURCE, prec=FP64, path=PATH_BATCHED,
               grid=None, kmax=16, penalty=0.0, want_images=False, refine=None, ctx=None):
    """chi^2 of every sample; image mode also returns nimg, nmissing (and
    img_xy (S, nsys, kmax, 2) when want_images).  refine = (max_iter, tol)
    refines every found image by Newton's method on the lens equation."""
    ctx = _ctx(ctx)
    dev = free_off.device
    S = int(free_off.numel()) - 1
    nsys = int(cat["off"].numel()) - 1
    chi2 = torch.empty(S, dtype=torch.float64, device=dev)
    res = dict(chi2=chi2)
    nimg = nmiss = img = None
    if mode == CHI2_IMAGE:
        nimg = torch.empty((S, nsys), dtype=torch.int32, device=dev)
        nmiss = torch.empty(S, dtype=torch.int32, device=dev)
        res.update(nimg=nimg, nmissing=nmiss)
        if want_images:
            img = torch.empty((S, nsys, kmax, 2), dtype=torch.float64, device=dev)
            res["img_xy"] = img
    B, K = _batch(fixed, free, free_off), _catalog(cat)
    O = _opts(mode, prec, path, grid, kmax, penalty, refine)
    st = lib().lens_chi2_batch(ctx.handle, C.byref(B), C.byref(K), C.byref(O), _ptr(chi2),
                               _ptr(nimg), _ptr(nmiss), _ptr(img), _stream(dev))
    if st == -4:
        res["overflow"] = True
        return res
    _check(st)
    res["overflow"] = False
    return res


def find_images(alpha, grid, src_x, src_y, f, kmax=16, ctx=None):
    """alpha: (2, ny, nx) float64 device tensor (Dls/Ds = 1).  Returns
    (nimg, tri, x, y) with per-source slot arrays (n_src, kmax)."""
    ctx = _ctx(ctx)
    dev = alpha.device
    assert alpha.dtype == torch.float64 and alpha.is_contiguous() and alpha.shape[0] == 2
    n = int(src_x.numel())
    nimg = torch.empty(n, dtype=torch.int32, device=dev)
    tri = torch.empty((n, kmax), dtype=torch.int64, device=dev)
    ix = torch.empty((n, kmax), dtype=torch.float64, device=dev)
    iy = torch.empty((n, kmax), dtype=torch.float64, device=dev)
    G = _grid(grid)
    nv = int(grid[0]) * int(grid[1])
    ay_ptr = alpha.data_ptr() + nv * 8
    st = lib().lens_find_images(ctx.handle, _ptr(alpha), C.c_void_p(ay_ptr), C.byref(G), n,
                                _ptr(src_x), _ptr(src_y), _ptr(f), int(kmax), _ptr(nimg),
                                _ptr(tri), _ptr(ix), _ptr(iy), _stream(dev))
    if st not in (0, -4):
        _check(st)
    return nimg, tri, ix, iy, st == -4


PLAN_FIXED_RESIDENT = 1


class Chi2Plan:
    """A lens_chi2_batch call (batched path) recorded into a HIP graph;
    launch() replays it on the current stream over the same buffers.
    resident=True: the fixed potentials and the catalogue are read once, at
    creation.  mode=CHI2_IMAGE records the image-plane pipeline (grid, kmax,
    penalty, refine as chi2_batch); nimg, nmissing (and img_xy when
    want_images) are then bound too, and status() reports what the last
    launch's search found (overflow, domain)."""

    def __init__(self, fixed, free, free_off, cat, prec=FP64, ctx=None, resident=False,
                 mode=CHI2_SOURCE, grid=None, kmax=16, penalty=0.0, want_images=False,
                 refine=None):
        self.ctx = _ctx(ctx)
        dev = free_off.device
        S = int(free_off.numel()) - 1
        nsys = int(cat["off"].numel()) - 1
        self.chi2 = torch.empty(S, dtype=torch.float64, device=dev)
        self.nimg = self.nmissing = self.img_xy = None
        if mode == CHI2_IMAGE:
            self.nimg = torch.empty((S, nsys), dtype=torch.int32, device=dev)
            self.nmissing = torch.empty(S, dtype=torch.int32, device=dev)
            if want_images:
                self.img_xy = torch.empty((S, nsys, kmax, 2), dtype=torch.float64, device=dev)
        self._keep = (fixed, free, free_off, cat)
        B, K = _batch(fixed, free, free_off), _catalog(cat)
        O = _opts(mode, prec, PATH_BATCHED, grid, kmax, penalty, refine)
        h = C.c_void_p()
        self.stream = torch.cuda.Stream(device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        _check(lib().lens_chi2_plan_create2(self.ctx.handle, C.byref(B), C.byref(K),
                                            C.byref(O), _ptr(self.chi2), _ptr(self.nimg),
                                            _ptr(self.nmissing), _ptr(self.img_xy),
                                            PLAN_FIXED_RESIDENT if resident else 0,
                                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().lens_chi2_plan_launch(self.handle, _stream(self.chi2.device)))
        return self.chi2

    def status(self):
        """Outcome of the last launch: False, or True when image slots
        overflowed; raises LensError for the search's domain errors."""
        st = lib().lens_chi2_plan_status(self.handle, _stream(self.chi2.device))
        if st == -4:
            return True
        _check(st)
        return False

    def close(self):
        if getattr(self, "handle", None):
            lib().lens_chi2_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mcmc:
    """Metropolis sampler over the free potentials' physical parameters.
    params (W, nfree, 7) FP64, updated in place; lo/hi/step (nfree, 7); u
    (W, 7 nfree + 1) uniforms in (0, 1], refilled by the caller before each
    step().  chi2 (W,) and accepted (W,) int32 are owned here."""

    def __init__(self, fixed, cat, params, lo, hi, step, u, convention=0, ctx=None):
        self.ctx = _ctx(ctx)
        dev = params.device
        W, nf = int(params.shape[0]), int(params.shape[1])
        for t in (params, lo, hi, step, u):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.device == dev
        assert params.shape[2] == 7 and lo.shape == hi.shape == step.shape == (nf, 7)
        assert u.shape == (W, 7 * nf + 1)
        self.params, self.u = params, u
        self.chi2 = torch.empty(W, dtype=torch.float64, device=dev)
        self.accepted = torch.zeros(W, dtype=torch.int32, device=dev)
        self._keep = (fixed, cat, lo, hi, step)
        D = _McmcDesc(W, nf, params.data_ptr(), self.chi2.data_ptr(), self.accepted.data_ptr(),
                      lo.data_ptr(), hi.data_ptr(), step.data_ptr(), u.data_ptr(),
                      int(convention))
        T, K = _pot(fixed), _catalog(cat)
        h = C.c_void_p()
        self.stream = torch.cuda.Stream(device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        _check(lib().lens_mcmc_create(self.ctx.handle, C.byref(T), C.byref(K), C.byref(D),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def step(self):
        _check(lib().lens_mcmc_step(self.handle, _stream(self.params.device)))

    def close(self):
        if getattr(self, "handle", None):
            lib().lens_mcmc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- host helpers -----------------------------------------------------------
def dlsds(zl, zs, om=0.3, ol=0.7):
    out = C.c_double()
    _check(lib().lens_dlsds(float(zl), float(zs), float(om), float(ol), C.byref(out)))
    return out.value


def b0_from_sigma(sigma, convention=0):
    out = C.c_double()
    _check(lib().lens_b0_from_sigma(float(sigma), int(convention), C.byref(out)))
    return out.value


def eps_from_e(e):
    out = C.c_double()
    _check(lib().lens_eps_from_e(float(e), C.byref(out)))
    return out.value


def catalog_with_dlsds(cat, zl, om=0.3, ol=0.7):
    """Catalogue dict (numpy) with f = Dls/Ds per system from its source redshift."""
    out = dict(cat)
    out["f"] = [dlsds(zl, z, om, ol) for z in cat["zs"]]
    return out
