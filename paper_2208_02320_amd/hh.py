"""Python binding of the C ABI in include/hh.h (ctypes; argument marshalling only).

Every step of the computation runs in the HIP library ``libhh.so``; this
module only converts arguments.  PyTorch supplies device memory (CUDA/HIP
tensors are passed by ``data_ptr()``) and the stream (the current torch
stream unless another is given).  Importing it without the built library,
or calling it without a gfx950 GPU, raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

HH_OK = 0
ERRORS = {
    -1: "HH_EINVAL", -2: "HH_EUNSUPPORTED", -3: "HH_ENOMEM", -4: "HH_EDEVICE",
    -5: "HH_ESINGULAR", -6: "HH_ENOCONV", -7: "HH_ESTAGNATED", -8: "HH_EBREAKDOWN",
}
KERNEL_CLASSES = ("zinv", "yinv", "x", "yfwd", "zfwd", "fin", "setup", "other")
NKERNEL = len(KERNEL_CLASSES)

# Exported symbols (checked by the CPU test suite against include/hh.h).
SYMBOLS = ("hh_default_opts", "hh_create", "hh_set_stream", "hh_destroy", "hh_last_error",
           "hh_workspace_bytes", "hh_release_workspace", "hh_size_supported", "hh_homogenize",
           "hh_homogenize_noalloc", "hh_homogenize_aniso", "hh_homogenize_batch", "hh_hierarchical", "hh_hierarchical_levels",
           "hh_gather_subimages",
           "hh_net_create", "hh_net_destroy", "hh_net_num_params", "hh_net_load", "hh_net_info", "hh_net_get_params",
           "hh_net_set_params", "hh_net_set_scaling", "hh_net_get_scaling", "hh_net_set_fraction_scaling", "hh_net_set_fraction_gate",
           "hh_net_set_interface_stats", "hh_net_get_interface_stats",
           "hh_net_get_fraction_scaling", "hh_net_forward", "hh_set_surrogate", "hh_plan_cache",
           "hh_net_gradient", "hh_net_train_step", "hh_net_predict", "hh_hierarchical_surrogate",
           "hh_richardson", "hh_moduli", "hh_mean_moduli")


class HHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "HH_E?"), code, msg))
        self.code = code


class Phase(ct.Structure):
    _fields_ = [("K", ct.c_double), ("G", ct.c_double)]


class Opts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("max_iter", ct.c_int), ("scheme", ct.c_int),
                ("precision", ct.c_int), ("nyquist", ct.c_int), ("profile", ct.c_int),
                ("stall_limit", ct.c_int), ("chunk", ct.c_int),
                ("ref_lambda", ct.c_double), ("ref_mu", ct.c_double),
                ("tune", ct.c_int), ("graph", ct.c_int), ("plan", ct.c_int * 3), ("loads_per_wave", ct.c_int),
                ("retry", ct.c_int), ("verify", ct.c_int), ("lanes", ct.c_int)]


class Report(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters", ct.c_int * 6), ("rel_resid", ct.c_double * 6),
                ("asym", ct.c_double), ("seconds", ct.c_double), ("voxel_iters", ct.c_double),
                ("items", ct.c_longlong), ("kernel_ms", ct.c_double * NKERNEL),
                ("kernel_launches", ct.c_int * NKERNEL), ("plan", ct.c_int * 3), ("setup_ms", ct.c_double),
                ("retried", ct.c_longlong), ("bytes_moved", ct.c_double), ("err_vs_oracle", ct.c_double)]

    def as_dict(self):
        return dict(status=self.status, iters=list(self.iters), rel_resid=list(self.rel_resid),
                    asym=self.asym, seconds=self.seconds, voxel_iters=self.voxel_iters,
                    items=self.items, plan=list(self.plan), setup_ms=self.setup_ms,
                    retried=self.retried, bytes_moved=self.bytes_moved, err_vs_oracle=self.err_vs_oracle,
                    kernel_ms={k: self.kernel_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
                    kernel_launches={k: self.kernel_launches[i] for i, k in enumerate(KERNEL_CLASSES)})


_lib = None


def load_library(path=LIB_PATH):
    """Load libhh.so (built by ``python -m paper_2208_02320_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is not built; run python -m paper_2208_02320_amd.build" % path)
    # torch first: its HIP runtime is then the one the library binds to (the
    # contexts run on torch's streams), never a second copy next to it
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(path)
    P, I, D, LL = ct.c_void_p, ct.c_int, ct.c_double, ct.c_longlong
    DP = ct.POINTER(ct.c_double)
    lib.hh_default_opts.argtypes = [ct.POINTER(Opts)]
    lib.hh_default_opts.restype = None
    lib.hh_create.argtypes = [ct.POINTER(P), I, P]
    lib.hh_set_stream.argtypes = [P, P]
    lib.hh_destroy.argtypes = [P]
    lib.hh_destroy.restype = None
    lib.hh_last_error.argtypes = [P]
    lib.hh_last_error.restype = ct.c_char_p
    lib.hh_workspace_bytes.argtypes = [P]
    lib.hh_workspace_bytes.restype = LL
    lib.hh_release_workspace.argtypes = [P]
    lib.hh_release_workspace.restype = None
    lib.hh_size_supported.argtypes = [I, I]
    lib.hh_homogenize.argtypes = [P, P, I, I, I, I, ct.POINTER(Phase), I, DP, ct.POINTER(I),
                                  ct.POINTER(Opts), DP, DP, ct.POINTER(Report)]
    lib.hh_homogenize_noalloc.argtypes = [P, P, I, I, I, ct.POINTER(Phase), I, ct.POINTER(Opts), DP,
                                          ct.POINTER(Report)]
    lib.hh_homogenize_aniso.argtypes = [P, P, I, I, I, I, ct.POINTER(Opts), DP, DP, ct.POINTER(Report)]
    lib.hh_homogenize_batch.argtypes = [P, I, ct.POINTER(I), P, LL, I, ct.POINTER(LL), ct.POINTER(Phase),
                                        ct.POINTER(I), ct.POINTER(I), ct.POINTER(I), ct.POINTER(Opts),
                                        DP, DP, ct.POINTER(I), ct.POINTER(I), ct.POINTER(Report)]
    lib.hh_hierarchical.argtypes = [P, P, I, I, I, I, ct.POINTER(Phase), I, I, I, I, ct.POINTER(Opts),
                                    DP, DP, ct.POINTER(Report)]
    lib.hh_hierarchical_levels.argtypes = [P, P, I, I, I, I, ct.POINTER(Phase), I, ct.POINTER(I), ct.POINTER(I), I,
                                           ct.POINTER(Opts), DP, ct.POINTER(Report)]
    lib.hh_gather_subimages.argtypes = [P, P, I, I, I, I, I, I, P]
    FP = ct.POINTER(ct.c_float)
    lib.hh_net_create.argtypes = [P, I, I, ct.c_ulonglong, ct.POINTER(P)]
    lib.hh_net_destroy.argtypes = [P]
    lib.hh_net_destroy.restype = None
    lib.hh_net_num_params.argtypes = [P]
    lib.hh_net_num_params.restype = LL
    lib.hh_net_load.argtypes = [P, ct.c_char_p, ct.POINTER(P)]
    lib.hh_net_info.argtypes = [P, ct.POINTER(I), ct.POINTER(I)]
    lib.hh_net_get_params.argtypes = [P, P, FP, LL]
    lib.hh_net_set_params.argtypes = [P, P, FP, LL]
    lib.hh_net_set_scaling.argtypes = [P, P, DP, DP]
    lib.hh_net_get_scaling.argtypes = [P, DP, DP]
    lib.hh_net_set_fraction_scaling.argtypes = [P, P, DP, DP]
    lib.hh_net_set_fraction_gate.argtypes = [P, P, D]
    lib.hh_net_set_interface_stats.argtypes = [P, P, D, D]
    lib.hh_net_get_interface_stats.argtypes = [P, DP, DP]
    lib.hh_net_get_fraction_scaling.argtypes = [P, DP, DP]
    lib.hh_net_forward.argtypes = [P, P, P, I, I, I, I, FP]
    lib.hh_net_gradient.argtypes = [P, P, P, I, I, I, I, FP, FP, FP]
    lib.hh_net_train_step.argtypes = [P, P, P, I, I, I, I, P, I, ct.c_float, FP]
    lib.hh_net_predict.argtypes = [P, P, P, I, I, I, I, DP]
    lib.hh_hierarchical_surrogate.argtypes = [P, P, I, I, I, I, ct.POINTER(Phase), I, I, I, P, P, D, D,
                                              ct.POINTER(Opts), DP, DP, ct.POINTER(I), ct.POINTER(Report)]
    lib.hh_set_surrogate.argtypes = [P, P, P, D, D]
    lib.hh_plan_cache.argtypes = [P, ct.c_char_p]
    lib.hh_richardson.argtypes = [ct.POINTER(I), DP, I, DP, DP]
    lib.hh_moduli.argtypes = [DP, DP, DP]
    lib.hh_mean_moduli.argtypes = [DP, LL, DP, DP]
    for name in SYMBOLS:
        getattr(lib, name)
    _lib = lib
    return lib


def default_opts(**kw):
    lib = load_library()
    o = Opts()
    lib.hh_default_opts(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        if k == "plan":
            v = (ct.c_int * 3)(*[int(x) for x in v])
        setattr(o, k, v)
    return o


def _dptr(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _fptr(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_float))


def _phases(phases):
    arr = (Phase * len(phases))()
    for i, (K, G) in enumerate(phases):
        arr[i].K, arr[i].G = float(K), float(G)
    return arr


def size_supported(n, precision=0):
    return bool(load_library().hh_size_supported(int(n), int(precision)))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _buffer(x, dtype):
    """(pointer, on_device, keepalive) for a torch tensor or array-like."""
    if _is_torch(x):
        import torch
        want = {np.uint8: torch.uint8, np.float64: torch.float64, np.float32: torch.float32}[dtype]
        if x.dtype != want:
            raise TypeError("expected a %s tensor" % want)
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ct.c_void_p(x.data_ptr()), int(x.is_cuda), x
    a = np.ascontiguousarray(np.asarray(x), dtype=dtype)
    return a.ctypes.data_as(ct.c_void_p), 0, a


@dataclass
class Result:
    C: np.ndarray
    C_raw: np.ndarray | None
    report: dict


class Context:
    """A library context bound to one device and stream."""

    def __init__(self, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs a gfx950 device")
        self._lib = load_library()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        h = ct.c_void_p()
        rc = self._lib.hh_create(ct.byref(h), self.device, ct.c_void_p(stream.cuda_stream))
        if rc != HH_OK:
            raise HHError(rc, self._lib.hh_last_error(None).decode() or "hh_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        self._stream = stream
        self._lib.hh_set_stream(self._h, ct.c_void_p(stream.cuda_stream))

    def _check(self, rc, allow=()):
        if rc != HH_OK and rc not in allow:
            raise HHError(rc, self._lib.hh_last_error(self._h).decode())
        return rc

    def workspace_bytes(self):
        return self._lib.hh_workspace_bytes(self._h)

    def release_workspace(self):
        self._lib.hh_release_workspace(self._h)

    def homogenize(self, labels, phases, loads=None, region=None, check=True, **opts):
        """C (6x6 Voigt, symmetrized), raw C, report for one label image [z][y][x]."""
        nz, ny, nx = tuple(labels.shape)
        ptr, dev, keep = _buffer(labels, np.uint8)
        o = default_opts(**opts)
        ph = _phases(phases)
        C = np.zeros(36)
        Craw = np.zeros(36)
        rep = Report()
        ld = None if loads is None else np.ascontiguousarray(np.asarray(loads, dtype=np.float64).T)
        rg = None if region is None else (ct.c_int * 6)(*[int(v) for v in region])
        rc = self._lib.hh_homogenize(self._h, ptr, nx, ny, nz, dev, ph, len(phases),
                                     None if ld is None else _dptr(ld), rg, ct.byref(o),
                                     _dptr(C), _dptr(Craw), ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return Result(C.reshape(6, 6), Craw.reshape(6, 6), rep.as_dict())

    def homogenize_noalloc(self, labels, phases, check=True, **opts):
        """hh_homogenize_noalloc: C (6x6, symmetrized) and report of one label
        image already on the device (a contiguous uint8 tensor [z][y][x])."""
        if not (_is_torch(labels) and labels.is_cuda):
            raise ValueError("labels must be a device tensor")
        nz, ny, nx = tuple(labels.shape)
        ptr, dev, keep = _buffer(labels, np.uint8)
        o = default_opts(**opts)
        ph = _phases(phases)
        C = np.zeros(36)
        rep = Report()
        rc = self._lib.hh_homogenize_noalloc(self._h, ptr, nx, ny, nz, ph, len(phases), ct.byref(o), _dptr(C),
                                             ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return Result(C.reshape(6, 6), None, rep.as_dict())

    def homogenize_aniso(self, C21, check=True, **opts):
        """Stiffness of an image of anisotropic voxels; C21 has shape (nz, ny, nx, 21)."""
        nz, ny, nx, k = tuple(C21.shape)
        if k != 21:
            raise ValueError("expected 21 components per voxel")
        ptr, dev, keep = _buffer(C21, np.float64)
        o = default_opts(**opts)
        C = np.zeros(36)
        Craw = np.zeros(36)
        rep = Report()
        rc = self._lib.hh_homogenize_aniso(self._h, ptr, nx, ny, nz, dev, ct.byref(o), _dptr(C),
                                           _dptr(Craw), ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return Result(C.reshape(6, 6), Craw.reshape(6, 6), rep.as_dict())

    def homogenize_batch(self, images, phase_sets, regions=None, labels_pack=None, check=True,
                         **opts):
        """Independent images (arrays [z][y][x], or shapes with ``labels_pack`` a
        device uint8 tensor holding them back to back).  Returns
        (C[n,6,6], C_raw[n,6,6], status[n], iters[n,6], report)."""
        n = len(images)
        dims = np.zeros(3 * n, dtype=np.int32)
        off = np.zeros(n, dtype=np.int64)
        pos = 0
        shapes = []
        for i, im in enumerate(images):
            shp = tuple(im) if labels_pack is not None else tuple(np.asarray(im).shape)
            nz, ny, nx = shp
            dims[3 * i:3 * i + 3] = (nx, ny, nz)
            off[i] = pos
            pos += nx * ny * nz
            shapes.append(shp)
        if labels_pack is None:
            pack = np.concatenate([np.ascontiguousarray(np.asarray(im, dtype=np.uint8)).ravel()
                                   for im in images])
            ptr, dev, keep = _buffer(pack, np.uint8)
        else:
            ptr, dev, keep = _buffer(labels_pack, np.uint8)
            if labels_pack.numel() < pos:
                raise ValueError("label pack too small")
        flat = []
        poff = np.zeros(n, dtype=np.int32)
        nph = np.zeros(n, dtype=np.int32)
        for i, ps in enumerate(phase_sets):
            poff[i] = len(flat)
            nph[i] = len(ps)
            flat.extend(ps)
        ph = _phases(flat)
        rg = None
        if regions is not None:
            rg = np.ascontiguousarray(np.asarray(regions, dtype=np.int32).reshape(n * 6))
        o = default_opts(**opts)
        C = np.zeros(36 * n)
        Craw = np.zeros(36 * n)
        st = np.zeros(n, dtype=np.int32)
        it = np.zeros(6 * n, dtype=np.int32)
        rep = Report()
        IP = ct.POINTER(ct.c_int)
        rc = self._lib.hh_homogenize_batch(
            self._h, n, dims.ctypes.data_as(IP), ptr, ct.c_longlong(pos), dev,
            off.ctypes.data_as(ct.POINTER(ct.c_longlong)), ph, poff.ctypes.data_as(IP),
            nph.ctypes.data_as(IP), None if rg is None else rg.ctypes.data_as(IP), ct.byref(o),
            _dptr(C), _dptr(Craw), st.ctypes.data_as(IP), it.ctypes.data_as(IP), ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return C.reshape(n, 6, 6), Craw.reshape(n, 6, 6), st, it.reshape(n, 6), rep.as_dict()

    def plan_cache(self, path):
        """Persistent autotuner plans in the text file ``path`` (None stops appending)."""
        self._check(self._lib.hh_plan_cache(self._h, None if path is None else os.fsencode(os.fspath(path))))

    def set_surrogate(self, net_a, net_b=None, spread_tol=0.02, bound_tol=0.0):
        """Networks used by hierarchical(..., use_surrogate=True); None detaches."""
        self._sur = (net_a, net_b)  # kept alive while attached
        self._check(self._lib.hh_set_surrogate(self._h, None if net_a is None else net_a._h,
                                               None if net_b is None else net_b._h, float(spread_tol),
                                               float(bound_tol)))

    def hierarchical(self, labels, phases, n_sub, pad=0, check=True, use_surrogate=False, **opts):
        """Two-level hierarchical C*; returns (C*, C_sub[(N/n)^3, 21], report)."""
        nz, ny, nx = tuple(labels.shape)
        ptr, dev, keep = _buffer(labels, np.uint8)
        o = default_opts(**opts)
        ph = _phases(phases)
        m = (nx // n_sub) * (ny // n_sub) * (nz // n_sub) if n_sub > 0 else 0
        C = np.zeros(36)
        Cs = np.zeros(max(1, m) * 21)
        rep = Report()
        rc = self._lib.hh_hierarchical(self._h, ptr, nx, ny, nz, dev, ph, len(phases), int(n_sub),
                                       int(pad), int(bool(use_surrogate)), ct.byref(o), _dptr(C), _dptr(Cs),
                                       ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return C.reshape(6, 6), Cs[:21 * m].reshape(m, 21), rep.as_dict()

    def hierarchical_levels(self, labels, phases, levels, check=True, **opts):
        """Repeated coarse-graining: levels = [(n_1, pad_1), (n_2, pad_2), ...];
        returns (C*, report)."""
        nz, ny, nx = tuple(labels.shape)
        ptr, dev, keep = _buffer(labels, np.uint8)
        o = default_opts(**opts)
        ph = _phases(phases)
        ns = (ct.c_int * len(levels))(*[int(n) for n, _ in levels])
        ps = (ct.c_int * len(levels))(*[int(p) for _, p in levels])
        C = np.zeros(36)
        rep = Report()
        rc = self._lib.hh_hierarchical_levels(self._h, ptr, nx, ny, nz, dev, ph, len(phases), ns, ps, len(levels),
                                              ct.byref(o), _dptr(C), ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return C.reshape(6, 6), rep.as_dict()

    def gather_subimages(self, labels, n_sub, pad=0, out=None):
        """Padded subimage boxes of an image [z][y][x] as a device uint8 tensor
        of shape (blocks, n_sub + 2 pad, ...), blocks in C order."""
        import torch
        nz, ny, nx = tuple(labels.shape)
        b = n_sub + 2 * pad
        m = (nx // n_sub) * (ny // n_sub) * (nz // n_sub)
        if out is None:
            out = torch.empty((m, b, b, b), dtype=torch.uint8, device="cuda:%d" % self.device)
        elif out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or out.numel() < m * b ** 3:
            raise ValueError("out must be a contiguous device uint8 tensor of %d bytes" % (m * b ** 3))
        ptr, dev, keep = _buffer(labels, np.uint8)
        self._check(self._lib.hh_gather_subimages(self._h, ptr, nx, ny, nz, dev, int(n_sub), int(pad),
                                                  ct.c_void_p(out.data_ptr())))
        del keep
        return out

    def hierarchical_surrogate(self, labels, phases, n_sub, pad, net_a, net_b=None, spread_tol=0.05,
                               bound_tol=0.02, check=True, **opts):
        """Two-level C* with network subimage stiffnesses and FFT fallback;
        returns (C*, C_sub[(N/n)^3, 21], fallback flags, report)."""
        nz, ny, nx = tuple(labels.shape)
        ptr, dev, keep = _buffer(labels, np.uint8)
        o = default_opts(**opts)
        ph = _phases(phases)
        m = (nx // n_sub) * (ny // n_sub) * (nz // n_sub)
        C = np.zeros(36)
        Cs = np.zeros(max(1, m) * 21)
        fb = np.zeros(max(1, m), dtype=np.int32)
        rep = Report()
        rc = self._lib.hh_hierarchical_surrogate(
            self._h, ptr, nx, ny, nz, dev, ph, len(phases), int(n_sub), int(pad), net_a._h,
            None if net_b is None else net_b._h, float(spread_tol), float(bound_tol), ct.byref(o), _dptr(C),
            _dptr(Cs), fb.ctypes.data_as(ct.POINTER(ct.c_int)), ct.byref(rep))
        if check:
            self._check(rc)
        del keep
        return C.reshape(6, 6), Cs[:21 * m].reshape(m, 21), fb[:m].astype(bool), rep.as_dict()


class Net:
    """CNN surrogate of the subimage stiffness (one network on one context).

    Label inputs are ``batch`` boxes of edge ``box`` (an array or a device
    uint8 tensor of shape (batch, box, box, box)); the network reads the
    n^3 window at (offset, offset, offset) of each box."""

    def __init__(self, ctx, nphase, n, seed=0):
        self.ctx = ctx
        self._lib = ctx._lib
        self.n = int(n)
        self.nphase = int(nphase)
        h = ct.c_void_p()
        ctx._check(self._lib.hh_net_create(ctx._h, self.nphase, self.n, ct.c_ulonglong(seed), ct.byref(h)))
        self._h = h

    @classmethod
    def load(cls, ctx, path):
        """A network from a training-pipeline .npz file, read by the library
        (hh_net_load)."""
        h = ct.c_void_p()
        ctx._check(ctx._lib.hh_net_load(ctx._h, os.fsencode(os.fspath(path)), ct.byref(h)))
        net = cls.__new__(cls)
        net.ctx, net._lib, net._h = ctx, ctx._lib, h
        nph, n = ct.c_int(), ct.c_int()
        ctx._check(ctx._lib.hh_net_info(h, ct.byref(nph), ct.byref(n)))
        net.nphase, net.n = nph.value, n.value
        return net

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hh_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return int(self._lib.hh_net_num_params(self._h))

    def get_params(self):
        p = np.zeros(self.num_params, dtype=np.float32)
        self.ctx._check(self._lib.hh_net_get_params(self.ctx._h, self._h, _fptr(p), p.size))
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        self.ctx._check(self._lib.hh_net_set_params(self.ctx._h, self._h, _fptr(p), p.size))

    def set_scaling(self, mean, scale):
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float64).reshape(21))
        s = np.ascontiguousarray(np.asarray(scale, dtype=np.float64).reshape(21))
        self.ctx._check(self._lib.hh_net_set_scaling(self.ctx._h, self._h, _dptr(m), _dptr(s)))

    def get_scaling(self):
        m, s = np.zeros(21), np.zeros(21)
        rc = self._lib.hh_net_get_scaling(self._h, _dptr(m), _dptr(s))
        if rc != HH_OK:
            raise HHError(rc, "hh_net_get_scaling")
        return m, s

    def set_fraction_scaling(self, mean, scale):
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float64).reshape(8))
        s = np.ascontiguousarray(np.asarray(scale, dtype=np.float64).reshape(8))
        self.ctx._check(self._lib.hh_net_set_fraction_scaling(self.ctx._h, self._h, _dptr(m), _dptr(s)))

    def set_fraction_gate(self, z_max):
        """Limit of the gate's phase-fraction test (feature scales; 0: off)."""
        self.ctx._check(self._lib.hh_net_set_fraction_gate(self.ctx._h, self._h, float(z_max)))

    def set_interface_stats(self, mean, scale):
        """Training mean and inverse standard deviation of the windows'
        interface density (the gate's texture test; scale 0: off)."""
        self.ctx._check(self._lib.hh_net_set_interface_stats(self.ctx._h, self._h, float(mean), float(scale)))

    def get_interface_stats(self):
        m, s = ct.c_double(), ct.c_double()
        rc = self._lib.hh_net_get_interface_stats(self._h, ct.byref(m), ct.byref(s))
        if rc != HH_OK:
            raise HHError(rc, "hh_net_get_interface_stats failed")
        return m.value, s.value

    def get_fraction_scaling(self):
        m, s = np.zeros(8), np.zeros(8)
        rc = self._lib.hh_net_get_fraction_scaling(self._h, _dptr(m), _dptr(s))
        if rc != HH_OK:
            raise HHError(rc, "hh_net_get_fraction_scaling")
        return m, s

    def _labels(self, labels, offset):
        shp = tuple(labels.shape)
        if len(shp) == 3:
            shp = (1,) + shp
        batch, box = shp[0], shp[1]
        if shp[1:] != (box, box, box):
            raise ValueError("label boxes must be cubes")
        ptr, dev, keep = _buffer(labels, np.uint8)
        return ptr, dev, keep, int(batch), int(box), int(offset)

    def forward(self, labels, offset=0):
        """Normalized outputs (batch, 21), float32."""
        ptr, dev, keep, batch, box, off = self._labels(labels, offset)
        out = np.zeros((batch, 21), dtype=np.float32)
        self.ctx._check(self._lib.hh_net_forward(self.ctx._h, self._h, ptr, dev, batch, box, off, _fptr(out)))
        del keep
        return out

    def gradient(self, labels, target, offset=0):
        """(loss, gradient over all parameters) of the mean squared error."""
        ptr, dev, keep, batch, box, off = self._labels(labels, offset)
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float32).reshape(batch, 21))
        g = np.zeros(self.num_params, dtype=np.float32)
        loss = ct.c_float()
        self.ctx._check(self._lib.hh_net_gradient(self.ctx._h, self._h, ptr, dev, batch, box, off, _fptr(t),
                                                  ct.byref(loss), _fptr(g)))
        del keep
        return loss.value, g

    def train_step(self, labels, target, lr, offset=0):
        """One Adam step; returns the loss before the step.  ``target`` is a
        (batch, 21) float32 array or device tensor of normalized values."""
        ptr, dev, keep, batch, box, off = self._labels(labels, offset)
        tptr, tdev, tkeep = _buffer(target if _is_torch(target) else
                                    np.asarray(target, dtype=np.float32).reshape(batch, 21), np.float32)
        if (target.numel() if _is_torch(target) else np.size(target)) != batch * 21:
            raise ValueError("target must hold batch x 21 values")
        loss = ct.c_float()
        self.ctx._check(self._lib.hh_net_train_step(self.ctx._h, self._h, ptr, dev, batch, box, off, tptr, tdev,
                                                    ct.c_float(lr), ct.byref(loss)))
        del keep, tkeep
        return loss.value

    def predict(self, labels, offset=0):
        """Stiffness C21 in GPa (batch, 21), float64."""
        ptr, dev, keep, batch, box, off = self._labels(labels, offset)
        out = np.zeros((batch, 21))
        self.ctx._check(self._lib.hh_net_predict(self.ctx._h, self._h, ptr, dev, batch, box, off, _dptr(out)))
        del keep
        return out


def richardson(ns, Cs):
    """Fit M(n) = M_inf + slope / n entrywise; Cs has shape (m, 6, 6)."""
    lib = load_library()
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    Cs = np.ascontiguousarray(np.asarray(Cs, dtype=np.float64).reshape(len(ns), 36))
    Ci = np.zeros(36)
    sl = np.zeros(36)
    rc = lib.hh_richardson(ns.ctypes.data_as(ct.POINTER(ct.c_int)), _dptr(Cs), len(ns), _dptr(Ci),
                           _dptr(sl))
    if rc != HH_OK:
        raise HHError(rc, "hh_richardson: need >= 2 distinct positive sizes")
    return Ci.reshape(6, 6), sl.reshape(6, 6)


def moduli(C):
    """(K, G) of the Voigt isotropic projection of a 6x6 stiffness."""
    lib = load_library()
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(36))
    K, G = ct.c_double(), ct.c_double()
    rc = lib.hh_moduli(_dptr(C), ct.byref(K), ct.byref(G))
    if rc != HH_OK:
        raise HHError(rc, "hh_moduli")
    return K.value, G.value


def mean_moduli(C_sub21):
    """Arithmetic mean of the subimages' Voigt (K, G) (the AM comparator of
    Sec. 5), from the m x 21 upper-triangle stiffnesses of hh_hierarchical."""
    lib = load_library()
    c = np.ascontiguousarray(np.asarray(C_sub21, dtype=np.float64).reshape(-1, 21))
    K, G = ct.c_double(), ct.c_double()
    rc = lib.hh_mean_moduli(_dptr(c), c.shape[0], ct.byref(K), ct.byref(G))
    if rc != HH_OK:
        raise HHError(rc, "hh_mean_moduli")
    return K.value, G.value


def upper21(C):
    C = np.asarray(C)
    return np.array([C[i, j] for i in range(6) for j in range(i, 6)])
