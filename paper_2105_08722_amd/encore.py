"""ctypes binding of libencore (include/encore.h): argument marshalling only.

Every step of the estimator runs in the HIP library; this module converts numpy /
torch arrays to pointers and status codes to exceptions.  If the shared library is
missing, importing the binding fails loudly (there is no CPU fallback).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libencore.so")

OK = 0
EINVAL = -1
ESIZE = -2
ENOMEM = -3
EDEVICE = -4
EUNSUPPORTED = -5
EAGAIN = -6

PERIODIC = 0x1
ALLPARITY = 0x2
DMR = 0x4
NORMALIZE = 0x8
PREC_FP64 = 0x00
PREC_FP32 = 0x10
PREC_SPLITBF16 = 0x20
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "splitbf16": PREC_SPLITBF16}
DEBUG_FULLGRID = 0x100

# every symbol include/encore.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_D = ctypes.c_double
_SZ = ctypes.c_size_t
SIGNATURES = {
    "encore_last_error": (ctypes.c_char_p, []),
    "encore_version": (ctypes.c_char_p, []),
    "encore_create": (_I, [_I, ctypes.POINTER(_P)]),
    "encore_destroy": (_I, [_P]),
    "encore_build_grid": (_I, [_P, _P, _P, _I64, _I64, _P, _D, _U32, _P, ctypes.POINTER(_P)]),
    "encore_build_grid_device": (_I, [_P, _P, _P, _I64, _I64, _P, _D, _U32, _P, ctypes.POINTER(_P)]),
    "encore_free_grid": (_I, [_P]),
    "encore_grid_size": (_I64, [_P]),
    "encore_npcf": (_I, [_P, _P, _I, _I, _I, _P, _U32, _D, _P, _SZ, _P, _I64, _P]),
    "encore_npcf_noalloc": (_I, [_P, _P, _I, _I, _I, _P, _U32, _D, _P, _SZ, _P, _I64, _P]),
    "encore_npcf_mesh": (_I, [_P, _P, _I, _D, _I, _I, _I, _P, _U32, _P, _SZ, _P]),
    "encore_npcf_batch": (_I, [_P, _P, _I, _I, _I, _I, _P, _U32, _P, _SZ, _P, _P, _P]),
    "encore_npcf_splits": (_I, [_P, _P, _P, _I, _I, _I, _I, _P, _U32, _D, _P, _SZ, _P, _SZ, _P]),
    "encore_npcf_simple": (_I, [_P, _P, _I64, _I, _I, _I, _P, _P, _U32, _P, _SZ]),
    "encore_num_multiplets": (_I64, [_I, _I, _U32]),
    "encore_num_bin_tuples": (_I64, [_I, _I]),
    "encore_multiplet_table": (_I, [_I, _I, _U32, _P, _SZ]),
    "encore_coupling_terms": (_I, [_I, _I, _U32, ctypes.POINTER(_I64), _I64, _P, _P, _P, _P]),
    "encore_wigner3j": (_D, [_I, _I, _I, _I, _I, _I]),
    "encore_debug_alm": (_I, [_P, _P, _I, _I, _P, _U32, _P, _I64, _P]),
    "encore_last_timings": (_I, [_P, _P, _SZ]),
    "encore_server_create": (_I, [_P, _SZ, _I, _I, _I64, ctypes.POINTER(_P)]),
    "encore_server_submit": (_I, [_P, _P, _P, _I64, _I64, _P, _I, _I, _I, _P, _U32, ctypes.POINTER(_I64)]),
    "encore_server_wait": (_I, [_P, _I64, _D, _P, _SZ, _P]),
    "encore_server_stats": (_I, [_P, _P, _SZ]),
    "encore_server_destroy": (_I, [_P]),
    "encore_plan_create": (_I, [_P, _P, _I, _I, _I, _P, _U32, _D, ctypes.POINTER(_P)]),
    "encore_plan_execute": (_I, [_P, _P, _SZ]),
    "encore_plan_destroy": (_I, [_P]),
    "encore_mfma_plan_stats": (_I, [_I, _I, _I, _U32, _P, _SZ]),
    "encore_autotune": (_I, [_P, _P, _P, _I64, _I64, _P, _I, _I, _I, _P, _U32, _I64, _P, _SZ]),
    "encore_edge_correct": (_I, [_P, _I, _I, _I, _U32, _P, _P, _SZ, _I, _P, _SZ, _P, _SZ,
                                 ctypes.POINTER(_I64)]),
}

_lib = None


class EncoreError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("encore error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libencore.so (raises if it has not been built).

    torch is imported first: it ships its own HIP runtime under the same soname
    (libamdhip64.so.7), and the library must bind to that one so that torch's
    device pointers and streams and the library's kernels share one runtime."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        if not os.path.exists(LIB_PATH):
            raise ImportError("libencore.so is not built (run __graft_entry__.build() or "
                              "python paper_2105_08722_amd/build.py); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise EncoreError(rc, lib().encore_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def version():
    return lib().encore_version().decode()


def num_multiplets(npcf, lmax, allparity=False):
    r = lib().encore_num_multiplets(npcf, lmax, ALLPARITY if allparity else 0)
    if r < 0:
        _check(int(r))
    return int(r)


def num_bin_tuples(npcf, nbins):
    r = lib().encore_num_bin_tuples(npcf, nbins)
    if r < 0:
        _check(int(r))
    return int(r)


def multiplet_table(npcf, lmax, allparity=False):
    width = 2 if npcf == 3 else 2 * npcf - 5
    n = num_multiplets(npcf, lmax, allparity)
    out = np.zeros(n * width, dtype=np.int32)
    _check(lib().encore_multiplet_table(npcf, lmax, ALLPARITY if allparity else 0, _ptr(out), out.size))
    return out.reshape(n, width)


def coupling_terms(npcf, lmax, allparity=False):
    """Half-sum terms: (lam[nt], l[nt, N-1], m[nt, N-1], coef[nt])."""
    flags = ALLPARITY if allparity else 0
    nt = ctypes.c_int64(0)
    _check(lib().encore_coupling_terms(npcf, lmax, flags, ctypes.byref(nt), 0, None, None, None, None))
    n = nt.value
    k = npcf - 1
    lam = np.zeros(n, dtype=np.int32)
    l = np.zeros(n * k, dtype=np.int32)
    m = np.zeros(n * k, dtype=np.int32)
    coef = np.zeros(n)
    _check(lib().encore_coupling_terms(npcf, lmax, flags, ctypes.byref(nt), n, _ptr(lam), _ptr(l),
                                       _ptr(m), _ptr(coef)))
    return lam, l.reshape(n, k), m.reshape(n, k), coef


def wigner3j(j1, j2, j3, m1, m2, m3):
    return lib().encore_wigner3j(j1, j2, j3, m1, m2, m3)


class Context:
    """An encore_ctx on one HIP device."""

    def __init__(self, device=0):
        h = _P()
        _check(lib().encore_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle is not None and self.handle.value:
            _check(lib().encore_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def last_timings(self):
        out = np.zeros(6)
        _check(lib().encore_last_timings(self.handle, _ptr(out), 6))
        return dict(total_ms=out[0], gather_ms=out[1], couple_ms=out[2], contract_ms=out[3],
                    batches=int(out[4]), pairs=int(out[5]))


class Grid:
    """A device-resident cell grid (encore_grid)."""

    def __init__(self, ctx, handle, n):
        self.ctx = ctx
        self.handle = handle
        self.n = n

    def free(self):
        if self.handle is not None and self.handle.value:
            _check(lib().encore_free_grid(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def _box3(box):
    if box is None:
        return None
    return _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))


def build_grid(ctx, pos, w, r_max, box=None, n_data=None, stream=None):
    """encore_build_grid from host arrays.  n_data: D-R weighting (first n_data are data)."""
    pos = _f64(pos, (-1, 3))
    w = _f64(w, (-1,))
    flags = (PERIODIC if box is not None else 0) | (DMR if n_data is not None else 0)
    b = _box3(box)
    h = _P()
    _check(lib().encore_build_grid(ctx.handle, _ptr(pos), _ptr(w), len(w), int(n_data or 0), _ptr(b),
                                   float(r_max), flags, stream, ctypes.byref(h)))
    return Grid(ctx, h, len(w))


def build_grid_device(ctx, pos, w, r_max, box=None, n_data=None):
    """encore_build_grid_device from torch tensors on the GPU (float64, contiguous)."""
    import torch
    if pos.dtype != torch.float64 or w.dtype != torch.float64 or not pos.is_cuda:
        raise ValueError("pos and w must be float64 device tensors")
    pos = pos.contiguous()
    w = w.contiguous()
    flags = (PERIODIC if box is not None else 0) | (DMR if n_data is not None else 0)
    b = _box3(box)
    h = _P()
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    _check(lib().encore_build_grid_device(ctx.handle, ctypes.c_void_p(pos.data_ptr()),
                                          ctypes.c_void_p(w.data_ptr()), w.numel(), int(n_data or 0),
                                          _ptr(b), float(r_max), flags, ctypes.c_void_p(stream),
                                          ctypes.byref(h)))
    return Grid(ctx, h, w.numel())


def npcf(ctx, grid, N, lmax, edges, precision="fp32", allparity=False, normalize=False, volume=0.0,
         primaries=None, stream=None, noalloc=False):
    """encore_npcf: Z (or zeta with normalize) as float64 [n_multiplets, n_bin_tuples].
    noalloc: call encore_npcf_noalloc instead (no device allocation in the call)."""
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0) | (NORMALIZE if normalize else 0)
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins) if nbins >= 0 else 0
    out = np.zeros(max(nlam * nB, 1))
    prim = None
    nsub = 0
    if primaries is not None:
        prim = np.ascontiguousarray(primaries, dtype=np.int64)
        nsub = len(prim)
        if nsub == 0:
            prim = np.zeros(1, dtype=np.int64)
    fn = lib().encore_npcf_noalloc if noalloc else lib().encore_npcf
    _check(fn(ctx.handle, grid.handle, int(N), int(lmax), nbins, _ptr(edges), flags,
              float(volume), _ptr(out), out.size, _ptr(prim), nsub, stream))
    return out[:nlam * nB].reshape(nlam, nB)


def npcf_mesh(ctx, delta, box, N, lmax, edges, precision="fp64", allparity=False, stream=None):
    """encore_npcf_mesh: Z of a density field on a periodic mesh, float64
    [n_multiplets, n_bin_tuples].  delta: a float64 CUDA tensor [n, n, n] on the
    context's device (C order: delta[ix, iy, iz])."""
    import torch
    if not (isinstance(delta, torch.Tensor) and delta.is_cuda and delta.dtype == torch.float64):
        raise TypeError("delta must be a float64 CUDA tensor")
    if delta.dim() != 3 or not (delta.shape[0] == delta.shape[1] == delta.shape[2]):
        raise ValueError("delta must be [n, n, n]")
    delta = delta.contiguous()
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0)
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins)
    out = np.zeros(max(nlam * nB, 1))
    _check(lib().encore_npcf_mesh(ctx.handle, ctypes.c_void_p(delta.data_ptr()), int(delta.shape[0]),
                                  float(box), int(N), int(lmax), nbins, _ptr(edges), flags, _ptr(out),
                                  out.size, stream))
    return out[:nlam * nB].reshape(nlam, nB)


def mfma_plan_stats(N, lmax, nbins, allparity=False):
    """encore_mfma_plan_stats as a dict."""
    out = np.zeros(4, dtype=np.int64)
    _check(lib().encore_mfma_plan_stats(int(N), int(lmax), int(nbins), ALLPARITY if allparity else 0,
                                        _ptr(out), 4))
    return {"tiles_per_16": int(out[0]), "row_tiles_per_16": int(out[1]), "t_entries": int(out[2]),
            "dense_entries": int(out[3])}


def autotune(ctx, pos, w, N, lmax, edges, box=None, n_data=None, precision="fp32", n_sample=8192):
    """encore_autotune: pick the cell shape and gather bins-per-item for jobs like
    this one; returns the report as a dict."""
    pos = _f64(pos, (-1, 3))
    w = _f64(w, (-1,))
    edges = _f64(edges, (-1,))
    flags = (PRECISIONS[precision] | (PERIODIC if box is not None else 0) |
             (DMR if n_data is not None else 0))
    rep = np.zeros(5)
    _check(lib().encore_autotune(ctx.handle, _ptr(pos), _ptr(w), len(w), int(n_data or 0), _ptr(_box3(box)),
                                 int(N), int(lmax), len(edges) - 1, _ptr(edges), flags, int(n_sample),
                                 _ptr(rep), 5))
    return {"cell_divisor": rep[0], "x_subdivision": rep[1], "bins_per_item": int(rep[2]),
            "best_ms": rep[3], "default_ms": rep[4]}


class Plan:
    """encore_plan: the hot path over one grid recorded once into a HIP graph
    (create), then replayed (execute)."""

    def __init__(self, ctx, grid, N, lmax, edges, precision="fp32", allparity=False, normalize=False,
                 volume=0.0):
        edges = _f64(edges, (-1,))
        nbins = len(edges) - 1
        flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0) | (NORMALIZE if normalize else 0)
        self.shape = (num_multiplets(N, lmax, allparity), num_bin_tuples(N, nbins))
        self.handle = _P()
        _check(lib().encore_plan_create(ctx.handle, grid.handle, int(N), int(lmax), nbins, _ptr(edges),
                                        flags, float(volume), ctypes.byref(self.handle)))

    def execute(self):
        out = np.zeros(max(self.shape[0] * self.shape[1], 1))
        _check(lib().encore_plan_execute(self.handle, _ptr(out), out.size))
        return out[:self.shape[0] * self.shape[1]].reshape(self.shape)

    def destroy(self):
        if self.handle is not None and self.handle.value:
            _check(lib().encore_plan_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def npcf_batch(ctx, grids, N, lmax, edges, precision="fp32", allparity=False, normalize=False,
               primaries=None, stream=None):
    """encore_npcf_batch: Z for several catalogs, float64 [n_jobs, n_multiplets, n_bin_tuples].
    primaries: None (every point of every catalog), or one entry per job, each None
    (every point) or an index array of that job's primaries."""
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0) | (NORMALIZE if normalize else 0)
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins)
    nj = len(grids)
    handles = (_P * nj)(*[g.handle.value for g in grids])
    out = np.zeros(max(nj * nlam * nB, 1))
    subs = counts = None
    keep = []
    if primaries is not None:
        if len(primaries) != nj:
            raise ValueError("primaries needs one entry per job")
        subs = (_P * nj)()
        counts = (ctypes.c_int64 * nj)()
        for j, p in enumerate(primaries):
            if p is None:
                continue
            a = np.ascontiguousarray(p, dtype=np.int64).reshape(-1)
            counts[j] = a.size
            if a.size == 0:
                a = np.zeros(1, dtype=np.int64)   # a valid pointer for an empty subset
            keep.append(a)
            subs[j] = a.ctypes.data
    _check(lib().encore_npcf_batch(ctx.handle, ctypes.cast(handles, _P), nj, int(N), int(lmax), nbins,
                                   _ptr(edges), flags, _ptr(out), out.size,
                                   ctypes.cast(subs, _P) if subs is not None else None,
                                   ctypes.cast(counts, _P) if counts is not None else None, stream))
    return out[:nj * nlam * nB].reshape(nj, nlam, nB)


def npcf_splits(ctx, data_grid, split_grids, N, lmax, edges, precision="fp32", allparity=False,
                normalize=False, volume=0.0, return_splits=False, stream=None):
    """encore_npcf_splits: mean over random parts of the D-R multiplets, float64
    [n_multiplets, n_bin_tuples] (with return_splits, also [n_splits, ...] per part).
    data_grid: the data alone; split_grids: D + R_k with n_data = len(data)."""
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0) | (NORMALIZE if normalize else 0)
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins)
    ns = len(split_grids)
    handles = (_P * max(ns, 1))(*[g.handle.value for g in split_grids])
    out = np.zeros(max(nlam * nB, 1))
    per = np.zeros(max(ns * nlam * nB, 1)) if return_splits else None
    _check(lib().encore_npcf_splits(ctx.handle, data_grid.handle, ctypes.cast(handles, _P), ns, int(N),
                                    int(lmax), nbins, _ptr(edges), flags, float(volume), _ptr(out), out.size,
                                    _ptr(per) if per is not None else None, per.size if per is not None else 0,
                                    stream))
    z = out[:nlam * nB].reshape(nlam, nB)
    if return_splits:
        return z, per[:ns * nlam * nB].reshape(ns, nlam, nB)
    return z


def build_split_grids(ctx, data_pos, data_w, rand_pos, rand_w, split_sizes, r_max, box=None):
    """Grids for npcf_splits: the data alone, then data + each consecutive part of
    the randoms (split_sizes points each) with D-R weights.  Returns (data_grid,
    [split grids]); the caller frees them."""
    data_pos = _f64(data_pos, (-1, 3))
    data_w = _f64(data_w, (-1,))
    rand_pos = _f64(rand_pos, (-1, 3))
    rand_w = _f64(rand_w, (-1,))
    sizes = [int(x) for x in split_sizes]
    if sum(sizes) != len(rand_w) or any(x < 1 for x in sizes):
        raise ValueError("split_sizes must be >= 1 and add up to the number of randoms")
    nd = len(data_w)
    gd = build_grid(ctx, data_pos, data_w, r_max, box=box)
    grids = []
    try:
        o = 0
        for n in sizes:
            pos = np.concatenate([data_pos, rand_pos[o:o + n]])
            w = np.concatenate([data_w, rand_w[o:o + n]])
            grids.append(build_grid(ctx, pos, w, r_max, box=box, n_data=nd))
            o += n
    except Exception:
        for g in grids:
            g.free()
        gd.free()
        raise
    return gd, grids


def debug_alm(ctx, grid, lmax, edges, primaries, precision="fp64", full_launch=False):
    """encore_debug_alm: complex a~ [k, nbins, (lmax+1)(lmax+2)/2] of the given primaries
    (full_launch: gather every point in one launch, as encore_npcf does)."""
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    prim = np.ascontiguousarray(primaries, dtype=np.int64)
    nlm = (lmax + 1) * (lmax + 2) // 2
    out = np.zeros((len(prim), nbins, nlm, 2))
    _check(lib().encore_debug_alm(ctx.handle, grid.handle, int(lmax), nbins, _ptr(edges),
                                  PRECISIONS[precision] | (DEBUG_FULLGRID if full_launch else 0),
                                  _ptr(prim), len(prim), _ptr(out)))
    return out[..., 0] + 1j * out[..., 1]


def edge_correct(ctx, N, lmax, nbins, nmult, rmult, allparity=False, lmax_out=None,
                 return_coupling=False):
    """encore_edge_correct: edge-corrected zeta [nout, nB] from the multiplets of the
    data-minus-randoms field (nmult) and of the randoms (rmult), both [nlam, nB] as
    npcf returns them.  lmax_out (default lmax) keeps the multiplets with every
    principal ell <= lmax_out.  With return_coupling, also M [nB, nlam, nlam] and the
    number of bin tuples without a solution."""
    nm = _f64(nmult, (-1,))
    rm = _f64(rmult, (-1,))
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins)
    if nm.size != nlam * nB or rm.size != nlam * nB:
        raise ValueError("nmult and rmult must hold %d x %d values" % (nlam, nB))
    lo = lmax if lmax_out is None else int(lmax_out)
    nout = num_multiplets(N, lo, allparity) if 0 <= lo <= lmax else 0
    z = np.zeros(max(nout * nB, 1))
    M = np.zeros(max(nB * nlam * nlam, 1)) if return_coupling else None
    bad = _I64(0)
    _check(lib().encore_edge_correct(ctx.handle, int(N), int(lmax), int(nbins),
                                     ALLPARITY if allparity else 0, _ptr(nm), _ptr(rm), nm.size, lo,
                                     _ptr(z), z.size, _ptr(M), 0 if M is None else M.size,
                                     ctypes.byref(bad)))
    z = z[:nout * nB].reshape(nout, nB)
    if return_coupling:
        return z, M[:nB * nlam * nlam].reshape(nB, nlam, nlam), int(bad.value)
    return z


def npcf_simple(pos, w, N, lmax, edges, box=None, precision="fp32", allparity=False):
    """encore_npcf_simple: one-shot grid build + npcf on device 0."""
    pos = _f64(pos, (-1, 3))
    w = _f64(w, (-1,))
    edges = _f64(edges, (-1,))
    nbins = len(edges) - 1
    flags = PRECISIONS[precision] | (ALLPARITY if allparity else 0)
    nlam = num_multiplets(N, lmax, allparity)
    nB = num_bin_tuples(N, nbins)
    out = np.zeros(max(nlam * nB, 1))
    _check(lib().encore_npcf_simple(_ptr(pos), _ptr(w), len(w), int(N), int(lmax), nbins, _ptr(edges),
                                    _ptr(_box3(box)), flags, _ptr(out), out.size))
    return out[:nlam * nB].reshape(nlam, nB)


class Server:
    """encore_server: catalog jobs admitted by device-memory footprint and run with
    continuous batching on n_lanes concurrent streams."""

    STATS = ("submitted", "done", "failed", "queued", "admitted", "bytes_held", "peak_bytes_held",
             "primaries_run", "slices", "gather_ms", "couple_ms", "workspace_bytes")

    def __init__(self, ctx, hbm_budget, n_lanes=2, max_active=64, slice_rows=262144):
        self.ctx = ctx
        h = _P()
        _check(lib().encore_server_create(ctx.handle, int(hbm_budget), int(n_lanes), int(max_active),
                                          int(slice_rows), ctypes.byref(h)))
        self.handle = h
        self._shape = {}

    def submit(self, pos, w, N, lmax, edges, box=None, n_data=None, precision="fp32",
               allparity=False, normalize=False):
        pos = _f64(pos, (-1, 3))
        w = _f64(w, (-1,))
        edges = _f64(edges, (-1,))
        flags = (PRECISIONS[precision] | (ALLPARITY if allparity else 0) | (NORMALIZE if normalize else 0)
                 | (PERIODIC if box is not None else 0) | (DMR if n_data is not None else 0))
        b = _box3(box)
        jid = _I64(0)
        _check(lib().encore_server_submit(self.handle, _ptr(pos), _ptr(w), len(w), int(n_data or 0), _ptr(b),
                                          int(N), int(lmax), len(edges) - 1, _ptr(edges), flags,
                                          ctypes.byref(jid)))
        self._shape[jid.value] = (num_multiplets(N, lmax, allparity), num_bin_tuples(N, len(edges) - 1))
        return jid.value

    def wait(self, job_id, timeout=None):
        """(zeta [n_multiplets, n_bin_tuples], times {submit, admit, start, done} in s).
        Raises EncoreError (code EAGAIN when the timeout passes first)."""
        nlam, nB = self._shape[job_id]
        out = np.zeros(max(nlam * nB, 1))
        t = np.zeros(4)
        rc = lib().encore_server_wait(self.handle, int(job_id), -1.0 if timeout is None else float(timeout),
                                      _ptr(out), out.size, _ptr(t))
        if rc != EAGAIN:
            self._shape.pop(job_id, None)
        _check(rc)
        return out[:nlam * nB].reshape(nlam, nB), dict(zip(("submit", "admit", "start", "done"), t.tolist()))

    def stats(self):
        out = np.zeros(12)
        _check(lib().encore_server_stats(self.handle, _ptr(out), 12))
        return dict(zip(self.STATS, out.tolist()))

    def close(self):
        if self.handle is not None and self.handle.value:
            _check(lib().encore_server_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
