"""Python binding of libpbr (include/pbr.h): argument marshalling only.

Every function has the name of the C entry point it wraps and forwards to it
through ctypes; all computation happens in the HIP library.  Vectors may be

* torch tensors on the context's GPU (complex128, contiguous): passed by device
  pointer with on_device = 1 and ordered on the context stream.  A Context takes
  torch's current stream when that is not the default stream; under torch's
  default (null) stream, whose handle is 0, the library creates its own stream
  with default flags, which HIP orders against the null stream in issue order,
  so torch work issued before a call completes before its kernels and work issued
  after it waits for them.  Context.stream_handle() names the stream in use;
* numpy arrays (complex128 / float64, C-contiguous): passed by host pointer with
  on_device = 0.

If libpbr.so is missing the import fails loudly: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbr.so")

PBR_OK, PBR_EINVAL, PBR_EODDGRID, PBR_ENOMEM, PBR_EDEVICE, PBR_ENOCONV, PBR_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "PBR_OK", -1: "PBR_EINVAL", -2: "PBR_EODDGRID", -3: "PBR_ENOMEM",
                -4: "PBR_EDEVICE", -5: "PBR_ENOCONV", -6: "PBR_ESTATE"}


class PbrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("maxit_outer", ctypes.c_int), ("maxit_inner", ctypes.c_int),
                ("ncv", ctypes.c_int), ("precond", ctypes.c_int),
                ("check_every", ctypes.c_int), ("seed", ctypes.c_int),
                ("concurrent", ctypes.c_int), ("graphs", ctypes.c_int),
                ("warm_start", ctypes.c_int)]


class PbrStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("op_applies", ctypes.c_int),
                ("pcg_iters_total", ctypes.c_int), ("pcg_iters_max", ctypes.c_int),
                ("matvecs", ctypes.c_int), ("n_zero", ctypes.c_int),
                ("converged", ctypes.c_int), ("nev_block", ctypes.c_int * 4),
                ("pcg_avg", ctypes.c_double), ("max_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["nev_block"] = list(self.nev_block)
        return d


class PbrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_SIGS = {
    "pbr_opts_default": (None, [ctypes.POINTER(PbrOpts)]),
    "pbr_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _dp, ctypes.c_int, _vp]),
    "pbr_set_material": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "pbr_set_reference": (ctypes.c_int, [_vp, _dp, ctypes.c_double]),
    "pbr_set_palette": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pbr_material_palette": (ctypes.c_int, [_vp]),
    "pbr_set_stencil_shape": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "pbr_set_solve_width": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pbr_set_precond_passes": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pbr_default_shift": (ctypes.c_double, [_vp]),
    "pbr_block_dim": (ctypes.c_long, [_vp, ctypes.c_int]),
    "pbr_block_gather": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int]),
    "pbr_block_scatter": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int]),
    "pbr_apply": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double, _vp, _vp,
                                 ctypes.c_int]),
    "pbr_apply_blocks": (ctypes.c_int, [_vp, _dp, ctypes.c_double, _vp, _vp, ctypes.c_int]),
    "pbr_eig_grad": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _vp,
                                    ctypes.c_int, _vp, _vp, ctypes.c_int]),
    "pbr_precond": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double, _vp, _vp,
                                   ctypes.c_int]),
    "pbr_precond_noalloc": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double, _vp,
                                           _vp]),
    "pbr_solve": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double, _vp, _vp,
                                 ctypes.POINTER(PbrOpts), ctypes.POINTER(PbrStats),
                                 ctypes.c_int]),
    "pbr_eigs": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(PbrOpts), _dp, _vp, ctypes.c_int,
                                ctypes.POINTER(PbrStats)]),
    "pbr_eigs_merged": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(PbrOpts), _dp,
                                       ctypes.POINTER(PbrStats)]),
    "pbr_eigs_merged_vecs": (ctypes.c_int, [_vp, _dp, ctypes.c_int, ctypes.c_double,
                                            ctypes.POINTER(PbrOpts), _dp,
                                            ctypes.POINTER(ctypes.c_int), _vp, ctypes.c_int,
                                            ctypes.POINTER(PbrStats)]),
    "pbr_band_path": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.POINTER(PbrOpts), _dp,
                                     ctypes.POINTER(PbrStats)]),
    "pbr_band_paths": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_dp),
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.POINTER(PbrOpts), ctypes.POINTER(_dp),
                                      ctypes.POINTER(PbrStats)]),
    "pbr_stream": (_vp, [_vp]),
    "pbr_copy_probe": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_long]),
    "pbr_last_error": (ctypes.c_char_p, [_vp]),
    "pbr_destroy": (None, [_vp]),
    "pbr_host_heev": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp]),
    "pbr_host_palette": (ctypes.c_int, [ctypes.c_long, _dp, _dp, _dp,
                                        ctypes.POINTER(ctypes.c_ubyte)]),
    "pbr_host_merge": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(_dp), _dp]),
}


def lib():
    """Load libpbr.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python -m paper_2606_03599_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, status):
    if status != PBR_OK:
        msg = lib().pbr_last_error(ctx)
        raise PbrError(status, msg.decode() if msg else "")
    return status


def _is_torch(x):
    return type(x).__module__.split(".")[0] == "torch"


def _vec(x, dtype=np.complex128):
    """(pointer, on_device, keepalive) of a vector argument."""
    if _is_torch(x):
        import torch
        want = torch.complex128 if dtype == np.complex128 else torch.float64
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"expected a contiguous {want} tensor")
        if x.device.type != "cuda":
            raise TypeError("torch tensors must live on the GPU; pass numpy arrays for host data")
        return x.data_ptr(), 1, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, 0, a


def _same_place(*ons):
    if len(set(ons)) != 1:
        raise TypeError("mix of device tensors and host arrays in one call")
    return ons[0]


def _kappa(kappa):
    k = (ctypes.c_double * 3)(*[float(v) for v in kappa])
    return ctypes.cast(k, _dp), k


def pbr_opts_default() -> PbrOpts:
    o = PbrOpts()
    lib().pbr_opts_default(ctypes.byref(o))
    return o


def pbr_create(n1, n2, n3, A_lat=None, device=0, stream=None):
    """Returns an opaque context handle (int)."""
    h = _vp()
    keep = None
    if A_lat is None:
        ap = None
    else:
        keep = np.asfortranarray(np.asarray(A_lat, dtype=np.float64).reshape(3, 3)).ravel(order="F")
        keep = np.ascontiguousarray(keep)
        ap = keep.ctypes.data_as(_dp)
    st = lib().pbr_create(ctypes.byref(h), int(n1), int(n2), int(n3), ap, int(device),
                          _vp(stream) if stream else None)
    _check(None, st)
    return h.value


def pbr_destroy(ctx):
    lib().pbr_destroy(ctx)


def pbr_stream(ctx):
    """hipStream_t (as an int, 0 for the null stream) the context orders its work on."""
    return lib().pbr_stream(ctx) or 0


def pbr_copy_probe(ctx, src, dst):
    """Streaming device copy src -> dst (torch tensors on the GPU, same byte size)."""
    ps, os_, ks = _vec(src, np.float64)
    pd, od, kd = _vec(dst, np.float64)
    if not (os_ and od):
        raise TypeError("the copy probe takes device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _check(ctx, lib().pbr_copy_probe(ctx, ps, pd, int(nbytes)))


def pbr_last_error(ctx):
    m = lib().pbr_last_error(ctx)
    return m.decode() if m else ""


def pbr_set_material(ctx, C21, rho):
    pc, oc, kc = _vec(C21, np.float64)
    pr, orr, kr = _vec(rho, np.float64)
    _check(ctx, lib().pbr_set_material(ctx, pc, pr, _same_place(oc, orr)))


def pbr_set_reference(ctx, C21_ref, rho_ref):
    a = np.ascontiguousarray(np.asarray(C21_ref, dtype=np.float64).reshape(21))
    _check(ctx, lib().pbr_set_reference(ctx, a.ctypes.data_as(_dp), float(rho_ref)))


def pbr_default_shift(ctx):
    return lib().pbr_default_shift(ctx)


def pbr_set_palette(ctx, enable):
    _check(ctx, lib().pbr_set_palette(ctx, int(enable)))


def pbr_material_palette(ctx):
    return lib().pbr_material_palette(ctx)


def pbr_set_stencil_shape(ctx, ti, tj):
    _check(ctx, lib().pbr_set_stencil_shape(ctx, int(ti), int(tj)))


def pbr_set_solve_width(ctx, bi):
    _check(ctx, lib().pbr_set_solve_width(ctx, int(bi)))


def pbr_set_precond_passes(ctx, passes):
    _check(ctx, lib().pbr_set_precond_passes(ctx, int(passes)))


def pbr_block_dim(ctx, block):
    return int(lib().pbr_block_dim(ctx, int(block)))


def pbr_block_gather(ctx, block, full, blk):
    pf, of, kf = _vec(full)
    pb, ob, kb = _vec(blk)
    _check(ctx, lib().pbr_block_gather(ctx, int(block), pf, pb, _same_place(of, ob)))
    return kb


def pbr_block_scatter(ctx, block, blk, full):
    pb, ob, kb = _vec(blk)
    pf, of, kf = _vec(full)
    _check(ctx, lib().pbr_block_scatter(ctx, int(block), pb, pf, _same_place(ob, of)))
    return kf


def pbr_apply(ctx, kappa, block, s, x, y):
    kp, kk = _kappa(kappa)
    px, ox, kx = _vec(x)
    py, oy, ky = _vec(y)
    _check(ctx, lib().pbr_apply(ctx, kp, int(block), float(s), px, py, _same_place(ox, oy)))
    return ky


def pbr_apply_blocks(ctx, kappa, s, x, y):
    kp, kk = _kappa(kappa)
    px, ox, kx = _vec(x)
    py, oy, ky = _vec(y)
    _check(ctx, lib().pbr_apply_blocks(ctx, kp, float(s), px, py, _same_place(ox, oy)))
    return ky


def pbr_eig_grad(ctx, kappa, block, lam, weight, evecs, gC21, grho):
    """Adds sum_s weight[s] d lambda_s / d (C21, rho) to gC21 (n x 21) and grho
    (n); evecs holds the nvec eigenvectors one after another."""
    kp, kk = _kappa(kappa)
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(-1))
    w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64).reshape(-1))
    if lam.size != w.size or lam.size < 1:
        raise ValueError("lambda and weight must have the same positive length")
    pv, ov, kv = _vec(evecs)
    pc, oc, kc = _vec(gC21, np.float64)
    pr, orr, kr = _vec(grho, np.float64)
    _check(ctx, lib().pbr_eig_grad(ctx, kp, int(block), int(lam.size), lam.ctypes.data_as(_dp),
                                   w.ctypes.data_as(_dp), pv, ov, pc, pr, _same_place(oc, orr)))
    return kc, kr


def pbr_precond(ctx, kappa, block, shift, r, z):
    kp, kk = _kappa(kappa)
    pr, orr, kr = _vec(r)
    pz, oz, kz = _vec(z)
    _check(ctx, lib().pbr_precond(ctx, kp, int(block), float(shift), pr, pz,
                                  _same_place(orr, oz)))
    return kz


def pbr_precond_noalloc(ctx, kappa, block, shift, r, z):
    """pbr_precond without any allocation; r, z device tensors."""
    pr, orr, kr = _vec(r)
    pz, oz, kz = _vec(z)
    if not (orr and oz):
        raise TypeError("pbr_precond_noalloc takes device tensors only")
    kp, kk = _kappa(kappa)
    _check(ctx, lib().pbr_precond_noalloc(ctx, kp, int(block), float(shift), pr, pz))
    return z


def pbr_solve(ctx, kappa, block, shift, b, x, opts=None, raise_on_noconv=True):
    kp, kk = _kappa(kappa)
    pb, ob, kb = _vec(b)
    px, ox, kx = _vec(x)
    st = PbrStats()
    o = opts if opts is not None else pbr_opts_default()
    status = lib().pbr_solve(ctx, kp, int(block), float(shift), pb, px, ctypes.byref(o),
                             ctypes.byref(st), _same_place(ob, ox))
    if status != PBR_ENOCONV or raise_on_noconv:
        _check(ctx, status)
    return kx, st


def pbr_eigs(ctx, kappa, block, nev, shift=0.0, opts=None, evecs=None, raise_on_noconv=True):
    """Returns (evals numpy (nev,), stats, evecs or None)."""
    kp, kk = _kappa(kappa)
    ev = np.zeros(int(nev))
    st = PbrStats()
    o = opts if opts is not None else pbr_opts_default()
    pe, oe, ke = (None, 0, None) if evecs is None else _vec(evecs)
    status = lib().pbr_eigs(ctx, kp, int(block), int(nev), float(shift), ctypes.byref(o),
                            ev.ctypes.data_as(_dp), pe, oe, ctypes.byref(st))
    if status != PBR_ENOCONV or raise_on_noconv:
        _check(ctx, status)
    return ev, st, ke


def pbr_eigs_merged(ctx, kappa, nev, shift=0.0, opts=None, raise_on_noconv=True):
    kp, kk = _kappa(kappa)
    ev = np.zeros(int(nev))
    st = PbrStats()
    o = opts if opts is not None else pbr_opts_default()
    status = lib().pbr_eigs_merged(ctx, kp, int(nev), float(shift), ctypes.byref(o),
                                   ev.ctypes.data_as(_dp), ctypes.byref(st))
    if status != PBR_ENOCONV or raise_on_noconv:
        _check(ctx, status)
    return ev, st


def pbr_eigs_merged_vecs(ctx, kappa, nev, evecs, shift=0.0, opts=None, raise_on_noconv=True):
    """Returns (evals (nev,), blocks (nev,) int, stats, evecs); evecs holds nev
    block-layout vectors of pbr_block_dim(ctx, 0) complex (torch tensor on the
    GPU or numpy array), vector t in block blocks[t]."""
    kp, kk = _kappa(kappa)
    ev = np.zeros(int(nev))
    bl = np.zeros(int(nev), dtype=np.int32)
    st = PbrStats()
    o = opts if opts is not None else pbr_opts_default()
    pe, oe, ke = _vec(evecs)
    status = lib().pbr_eigs_merged_vecs(ctx, kp, int(nev), float(shift), ctypes.byref(o),
                                        ev.ctypes.data_as(_dp),
                                        bl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pe, oe,
                                        ctypes.byref(st))
    if status != PBR_ENOCONV or raise_on_noconv:
        _check(ctx, status)
    return ev, bl, st, ke


def pbr_band_path(ctx, kappas, nev, blocked=True, shift=0.0, opts=None, raise_on_noconv=True):
    ks = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64).reshape(-1, 3))
    ev = np.zeros((ks.shape[0], int(nev)))
    st = PbrStats()
    o = opts if opts is not None else pbr_opts_default()
    status = lib().pbr_band_path(ctx, ks.shape[0], ks.ctypes.data_as(_dp), int(nev),
                                 1 if blocked else 0, float(shift), ctypes.byref(o),
                                 ev.ctypes.data_as(_dp), ctypes.byref(st))
    if status != PBR_ENOCONV or raise_on_noconv:
        _check(ctx, status)
    return ev, st


def pbr_band_paths(ctxs, kappas_list, nev, blocked=True, shift=0.0, opts=None,
                   raise_on_noconv=True):
    """Band paths of several cells concurrently (one context per cell); returns
    ([evals per cell], [PbrStats per cell])."""
    ncells = len(ctxs)
    ks = [np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, 3))
          for k in kappas_list]
    evs = [np.zeros((k.shape[0], int(nev))) for k in ks]
    hs = (_vp * ncells)(*[c if isinstance(c, int) else c.value for c in ctxs])
    nks = (ctypes.c_int * ncells)(*[k.shape[0] for k in ks])
    kp = (_dp * ncells)(*[k.ctypes.data_as(_dp) for k in ks])
    ep = (_dp * ncells)(*[e.ctypes.data_as(_dp) for e in evs])
    sts = (PbrStats * ncells)()
    o = opts if opts is not None else pbr_opts_default()
    status = lib().pbr_band_paths(ncells, hs, nks, kp, int(nev), 1 if blocked else 0,
                                  float(shift), ctypes.byref(o), ep, sts)
    if status != PBR_OK and (status != PBR_ENOCONV or raise_on_noconv):
        bad = None
        for c in ctxs:
            if lib().pbr_last_error(c):
                bad = c
                break
        _check(bad, status)
    return evs, list(sts)


def pbr_host_heev(A):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128).T)  # column-major
    m = A.shape[0]
    w = np.zeros(m)
    V = np.zeros((m, m), dtype=np.complex128)
    st = lib().pbr_host_heev(m, A.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                             V.ctypes.data_as(_dp))
    if st != 0:
        raise PbrError(st, "pbr_host_heev failed")
    return w, np.ascontiguousarray(V.T)


def pbr_host_merge(nev, block_vals):
    nb = (ctypes.c_int * 4)(*[len(v) for v in block_vals])
    arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in block_vals]
    ptrs = (_dp * 4)(*[a.ctypes.data_as(_dp) for a in arrs])
    out = np.zeros(int(nev))
    mask = lib().pbr_host_merge(int(nev), nb, ptrs, out.ctypes.data_as(_dp))
    return mask, out


def pbr_host_palette(C21, rho):
    """(rows (k x 22), idx (n,) uint8) of the material's palette form, or None
    when it has more than 256 distinct rows."""
    C = np.ascontiguousarray(np.asarray(C21, dtype=np.float64))
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
    n = r.size
    if C.shape != (n, 21):
        raise ValueError("C21 must be n x 21 and rho n")
    rows = np.zeros((256, 22))
    idx = np.zeros(n, dtype=np.uint8)
    k = lib().pbr_host_palette(n, C.ctypes.data_as(_dp), r.ctypes.data_as(_dp),
                               rows.ctypes.data_as(_dp),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if k < 0:
        raise PbrError(k, "pbr_host_palette failed")
    return None if k == 0 else (rows[:k].copy(), idx)


def band_paths(contexts, kappas_list, nev, blocked=True, shift=0.0, opts=None):
    """pbr_band_paths over Context objects: cells of their own sizes, concurrently."""
    return pbr_band_paths([c.h for c in contexts], kappas_list, nev, blocked, shift, opts)


class Context:
    """Owning wrapper around a pbr_ctx handle (methods forward to the pbr_* calls)."""

    def __init__(self, dims, A_lat=None, device=0, stream=None):
        if isinstance(dims, int):
            dims = (dims, dims, dims)
        self.dims = tuple(int(d) for d in dims)
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                stream = None
        self.h = pbr_create(*self.dims, A_lat=A_lat, device=device, stream=stream)

    def stream_handle(self):
        """The hipStream_t the context launches on (events that time its kernels
        are recorded on this stream; see pbr_stream)."""
        return pbr_stream(self.h)

    def copy_probe(self, src, dst):
        pbr_copy_probe(self.h, src, dst)

    def close(self):
        if self.h:
            pbr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, C21, rho):
        pbr_set_material(self.h, C21, rho)

    def set_reference(self, C21_ref, rho_ref):
        pbr_set_reference(self.h, C21_ref, rho_ref)

    def default_shift(self):
        return pbr_default_shift(self.h)

    def set_palette(self, enable):
        """Let the kernels read the material's palette form (True) or the dense form."""
        pbr_set_palette(self.h, 1 if enable else 0)

    def palette_size(self):
        """Palette rows the kernels read; 0 for the dense form."""
        return pbr_material_palette(self.h)

    def set_stencil_shape(self, ti=0, tj=0):
        """Pin the operator kernel's tile shape (16 x 13, or 16 x 11 for the palette
        form); 0, 0 returns the choice to the autotuner."""
        pbr_set_stencil_shape(self.h, ti, tj)

    def set_solve_width(self, bi=0):
        """Pin the mode-solve pass's i-width (8, 16 or 32); 0 returns it to the
        autotuner."""
        pbr_set_solve_width(self.h, bi)

    def set_precond_passes(self, passes=0):
        """0 automatic (three passes for a block where available), 3 or 5."""
        pbr_set_precond_passes(self.h, passes)

    def block_dim(self, block):
        return pbr_block_dim(self.h, block)

    def apply(self, kappa, block, s, x, y):
        return pbr_apply(self.h, kappa, block, s, x, y)

    def apply_blocks(self, kappa, s, x, y):
        return pbr_apply_blocks(self.h, kappa, s, x, y)

    def eig_grad(self, kappa, block, lam, weight, evecs, gC21, grho):
        return pbr_eig_grad(self.h, kappa, block, lam, weight, evecs, gC21, grho)

    def precond(self, kappa, block, shift, r, z):
        return pbr_precond(self.h, kappa, block, shift, r, z)

    def precond_noalloc(self, kappa, block, shift, r, z):
        return pbr_precond_noalloc(self.h, kappa, block, shift, r, z)

    def solve(self, kappa, block, shift, b, x, opts=None):
        return pbr_solve(self.h, kappa, block, shift, b, x, opts)

    def eigs(self, kappa, block, nev, shift=0.0, opts=None, evecs=None):
        return pbr_eigs(self.h, kappa, block, nev, shift, opts, evecs)

    def eigs_merged(self, kappa, nev, shift=0.0, opts=None):
        return pbr_eigs_merged(self.h, kappa, nev, shift, opts)

    def eigs_merged_vecs(self, kappa, nev, evecs, shift=0.0, opts=None):
        return pbr_eigs_merged_vecs(self.h, kappa, nev, evecs, shift, opts)

    def band_path(self, kappas, nev, blocked=True, shift=0.0, opts=None):
        return pbr_band_path(self.h, kappas, nev, blocked, shift, opts)

    def gather(self, block, full, blk):
        return pbr_block_gather(self.h, block, full, blk)

    def scatter(self, block, blk, full):
        return pbr_block_scatter(self.h, block, blk, full)
