"""ctypes binding of libamigpu.so: argument marshalling only.

Names follow the C ABI (``include/amigpu.h``): :class:`Terms` wraps
``amiConstruct`` / ``amiTermsInfo`` / ``amiTermsCanonical`` / ``amiFree``;
:func:`evaluate` and :func:`evaluate_hubbard` wrap ``amiEvaluate`` and
``amiEvaluateHubbard``, passing device pointers of torch tensors and the
current torch stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libamigpu.so"

AMI_FACTORIZE = 1
AMI_MULTIPOLE = 2


def _flags(factorize: bool, multipole: bool) -> int:
    return (AMI_FACTORIZE if factorize else 0) | (AMI_MULTIPOLE if multipole else 0)

_STATUS = {0: "AMI_OK", -1: "AMI_E_ARG", -2: "AMI_E_LABEL", -3: "AMI_E_MULTIPOLE",
           -4: "AMI_E_COEFF", -5: "AMI_E_HIP", -6: "AMI_E_OOM", -7: "AMI_E_UNSUPPORTED"}


class AmiError(RuntimeError):
    """A non-AMI_OK status; ``.status`` holds the code name."""

    def __init__(self, code: int, msg: str):
        self.code = code
        self.status = _STATUS.get(code, str(code))
        super().__init__(f"{self.status}: {msg}")


_lib = None


class AmiBatchItem(ctypes.Structure):
    """Mirror of the C struct AmiBatchItem (include/amigpu.h)."""
    _fields_ = [("terms", ctypes.c_void_p), ("energies", ctypes.c_void_p),
                ("stride_s", ctypes.c_int64), ("stride_i", ctypes.c_int64),
                ("k", ctypes.c_void_p), ("stride_k", ctypes.c_int64),
                ("q", ctypes.c_double * 8), ("t", ctypes.c_double), ("mu", ctypes.c_double),
                ("n_e", ctypes.c_int64), ("ext_freqs", ctypes.c_void_p), ("n_f", ctypes.c_int64),
                ("beta", ctypes.c_double), ("e_reg", ctypes.c_double),
                ("out", ctypes.c_void_p), ("out_sum", ctypes.c_void_p)]


class AmiBatchTuning(ctypes.Structure):
    """Mirror of the C struct AmiBatchTuning."""
    _fields_ = [("block", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("tile_factor", ctypes.c_int32), ("kernels", ctypes.c_int32)]


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load libamigpu.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2311_17189_amd.build.build()")
    lib = ctypes.CDLL(path)
    c_i32, c_i64, c_u32, c_dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    vp = ctypes.c_void_p
    lib.amiConstruct.argtypes = [c_i32, c_i32, c_i32, c_i32, vp, vp, vp, c_u32, ctypes.POINTER(vp)]
    lib.amiConstruct.restype = c_i32
    lib.amiFree.argtypes = [vp]
    lib.amiFree.restype = None
    lib.amiTermsInfo.argtypes = [vp, vp]
    lib.amiTermsInfo.restype = c_i32
    lib.amiTermsCanonical.argtypes = [vp, c_i32, vp, c_i64, ctypes.POINTER(c_i64)]
    lib.amiTermsCanonical.restype = c_i32
    lib.amiTermsUpload.argtypes = [vp]
    lib.amiTermsUpload.restype = c_i32
    lib.amiEvaluate.argtypes = [vp, vp, c_i64, c_i64, c_i64, vp, c_i64, c_dbl, c_dbl, vp, vp, vp]
    lib.amiEvaluate.restype = c_i32
    lib.amiEvaluateComplex.argtypes = [vp, vp, c_i64, c_i64, c_i64, vp, c_i64, c_dbl, c_dbl, vp, vp, vp]
    lib.amiEvaluateComplex.restype = c_i32
    lib.amiSetTwoPassChunkBytes.argtypes = [c_i64]
    lib.amiSetTwoPassChunkBytes.restype = c_i32
    lib.amiEvaluateHubbard.argtypes = [vp, vp, c_i64, c_i64, vp, c_dbl, c_dbl, vp, c_i64, c_dbl,
                                       c_dbl, vp, vp, vp]
    lib.amiEvaluateHubbard.restype = c_i32
    lib.amiEvaluateAdjoint.argtypes = [vp, vp, c_i64, c_i64, c_i64, vp, c_i64, c_dbl, c_dbl, vp, vp,
                                       vp, vp, vp, vp, vp, vp]
    lib.amiEvaluateAdjoint.restype = c_i32
    lib.amiEvaluateComplexAdjoint.argtypes = lib.amiEvaluateAdjoint.argtypes
    lib.amiEvaluateComplexAdjoint.restype = c_i32
    lib.amiEvaluateHubbardAdjoint.argtypes = [vp, vp, c_i64, c_i64, vp, c_dbl, c_dbl, vp, c_i64, c_dbl,
                                              c_dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.amiEvaluateHubbardAdjoint.restype = c_i32
    lib.amiEvaluateHubbardAdjointNoAlloc.argtypes = lib.amiEvaluateHubbardAdjoint.argtypes
    lib.amiEvaluateHubbardAdjointNoAlloc.restype = c_i32
    lib.amiSetVariant.argtypes = [vp, c_i32]
    lib.amiSetVariant.restype = c_i32
    lib.amiReadGraph.argtypes = [ctypes.c_char_p, vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]
    lib.amiReadGraph.restype = c_i32
    lib.amiConstructGraph.argtypes = [c_i32, c_i32, vp, c_u32, ctypes.POINTER(vp)]
    lib.amiConstructGraph.restype = c_i32
    lib.amiTermsLabels.argtypes = [vp, vp, vp, vp]
    lib.amiTermsLabels.restype = c_i32
    lib.amiIntegrateHubbard.argtypes = [vp, c_i64, ctypes.c_uint64, vp, c_dbl, c_dbl, vp, c_i64, c_dbl, c_dbl,
                                        vp, vp]
    lib.amiIntegrateHubbard.restype = c_i32
    lib.amiTermsSpecialize.argtypes = [vp, c_i32]
    lib.amiTermsSpecialize.restype = c_i32
    lib.amiTermsSource.argtypes = [vp, c_i32, ctypes.c_char_p, c_i64, ctypes.POINTER(c_i64)]
    lib.amiTermsSource.restype = c_i32
    lib.amiBatchSource.argtypes = [vp, c_i32, vp, c_i32, c_i32, ctypes.c_char_p, c_i64, ctypes.POINTER(c_i64)]
    lib.amiBatchSource.restype = c_i32
    lib.amiMeasureFp64Peak.argtypes = [c_i64, ctypes.POINTER(ctypes.c_double), vp]
    lib.amiMeasureFp64Peak.restype = c_i32
    lib.amiKernelTimerStart.argtypes = [c_i32]
    lib.amiKernelTimerStart.restype = c_i32
    lib.amiKernelTimerStop.argtypes = [vp, c_i32, ctypes.POINTER(c_i32)]
    lib.amiKernelTimerStop.restype = c_i32
    lib.amiLastVariant.argtypes = []
    lib.amiLastVariant.restype = ctypes.c_char_p
    lib.amiBatchCreate.argtypes = [ctypes.POINTER(AmiBatchItem), c_i32, ctypes.POINTER(AmiBatchTuning),
                                   ctypes.POINTER(vp)]
    lib.amiBatchCreate.restype = c_i32
    lib.amiBatchRun.argtypes = [vp, vp]
    lib.amiBatchRun.restype = c_i32
    lib.amiBatchInfo.argtypes = [vp, vp]
    lib.amiBatchInfo.restype = c_i32
    lib.amiBatchFree.argtypes = [vp]
    lib.amiBatchFree.restype = None
    lib.amiLastError.argtypes = []
    lib.amiLastError.restype = ctypes.c_char_p
    lib.amiVersion.argtypes = []
    lib.amiVersion.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        msg = load_library().amiLastError().decode()
        raise AmiError(code, msg)


def version() -> str:
    return load_library().amiVersion().decode()


_timer_capacity = 0


def measure_fp64_peak(iters: int = 1 << 16, stream=None) -> float:
    """FP64 FMA throughput of the current device in TFLOP/s
    (``amiMeasureFp64Peak``; blocks until done)."""
    v = ctypes.c_double()
    _check(load_library().amiMeasureFp64Peak(int(iters), ctypes.byref(v), _stream_ptr(stream)))
    return v.value


def kernel_timer_start(capacity: int):
    """Record HIP events around the main kernel of the next ``capacity``
    evaluate/adjoint calls on this thread (``amiKernelTimerStart``)."""
    global _timer_capacity
    _check(load_library().amiKernelTimerStart(int(capacity)))
    _timer_capacity = int(capacity)


def kernel_timer_stop() -> list:
    """Durations (ms) of the recorded kernels, in call order (``amiKernelTimerStop``)."""
    lib = load_library()
    buf = (ctypes.c_float * max(_timer_capacity, 1))()
    n = ctypes.c_int32()
    _check(lib.amiKernelTimerStop(buf, max(_timer_capacity, 1), ctypes.byref(n)))
    return [float(buf[i]) for i in range(min(n.value, _timer_capacity))]


# kernel variants (amiSetVariant)
VARIANT_AUTO, VARIANT_TABLES, VARIANT_PACKED, VARIANT_SPECIALIZED, VARIANT_TWO_PASS = 0, 1, 2, 3, 4


def set_two_pass_chunk_bytes(nbytes: int):
    """``amiSetTwoPassChunkBytes``: bound on one chunk of the two-pass workspace."""
    _check(load_library().amiSetTwoPassChunkBytes(int(nbytes)))


def last_variant() -> str:
    """Kernel variant launched by the last evaluate call on this thread."""
    return load_library().amiLastVariant().decode()


class Terms:
    """Symbolic AMI solution of one integrand (``amiConstruct``).

    ``alpha`` int [nG, nF] (summed slots first, external last), ``eps`` int
    [nG, nE], ``n_int`` number of sums, ``fermionic`` optional 0/1 [nF].
    """

    def __init__(self, alpha, eps, n_int: int, fermionic=None, factorize: bool = False, multipole: bool = False):
        lib = load_library()
        a = np.ascontiguousarray(np.asarray(alpha, dtype=np.int8))
        e = np.ascontiguousarray(np.asarray(eps, dtype=np.int8))
        if a.ndim != 2 or e.ndim != 2:
            raise AmiError(-1, "alpha and eps must be 2-D")
        f = None
        if fermionic is not None:
            f = np.ascontiguousarray(np.asarray(fermionic, dtype=np.uint8).reshape(-1))
        h = ctypes.c_void_p()
        code = lib.amiConstruct(a.shape[0], e.shape[1], a.shape[1], int(n_int),
                                a.ctypes.data, e.ctypes.data,
                                None if f is None else f.ctypes.data,
                                _flags(factorize, multipole), ctypes.byref(h))
        _check(code)
        self._h = h
        self.n_g, self.n_freq = a.shape
        self.n_eps = e.shape[1]
        self.n_int = int(n_int)
        self.alpha = a
        self.eps = e

    @classmethod
    def from_graph(cls, edges, n_vertices: Optional[int] = None, factorize: bool = False,
                   multipole: bool = False) -> "Terms":
        """``amiConstructGraph``: ``edges`` int [n, 4] rows (source, target, B/F, spin)
        of a Feynman graph (Sec. 2.5), labelled and constructed by the library."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 4))
        nv = int(e[:, :2].max()) + 1 if n_vertices is None else int(n_vertices)
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        _check(load_library().amiConstructGraph(nv, e.shape[0], e.ctypes.data, _flags(factorize, multipole),
                                                ctypes.byref(self._h)))
        self.alpha, self.eps, self.fermionic = self.labels()
        self.n_g, self.n_freq = self.alpha.shape
        self.n_eps = self.eps.shape[1]
        self.n_int = self.info()["n_int"]
        return self

    @classmethod
    def from_graph_file(cls, path: str, factorize: bool = False, multipole: bool = False) -> "Terms":
        """Read a 4-column graph file (``amiReadGraph``) and construct it."""
        return cls.from_graph(read_graph(path), factorize=factorize, multipole=multipole)

    def labels(self):
        """R0 of the handle (``amiTermsLabels``): alpha int8 [n_g, n_freq], eps int8
        [n_g, n_eps], fermionic uint8 [n_freq]."""
        inf = self.info()
        n_g = inf["n_g"]
        alpha = np.zeros((n_g, inf["n_freq"]), dtype=np.int8)
        eps = np.zeros((n_g, inf["n_eps"]), dtype=np.int8)
        ferm = np.zeros(inf["n_freq"], dtype=np.uint8)
        _check(load_library().amiTermsLabels(self._h, alpha.ctypes.data, eps.ctypes.data, ferm.ctypes.data))
        return alpha, eps, ferm

    @classmethod
    def from_diagram(cls, d, factorize: bool = False, multipole: bool = False) -> "Terms":
        return cls(d.alpha, d.eps, d.n_int, d.fermionic, factorize, multipole)

    @property
    def handle(self) -> int:
        return self._h.value

    def info(self) -> dict:
        buf = np.zeros(16, dtype=np.int64)
        _check(load_library().amiTermsInfo(self._h, buf.ctypes.data))
        keys = ["T", "n_int", "n_eps", "n_freq", "n_ext", "L", "D", "G", "tree_nodes",
                "raw_terms", "leaves_per_term", "dens_per_term", "packable", "products", "n_g", "uniform"]
        return {k: int(buf[i]) for i, k in enumerate(keys)}

    def canonical(self, from_tree: bool = False) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_int64()
        _check(lib.amiTermsCanonical(self._h, int(from_tree), None, 0, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.int32)
        _check(lib.amiTermsCanonical(self._h, int(from_tree), buf.ctypes.data, n.value, ctypes.byref(n)))
        return buf

    def upload(self):
        _check(load_library().amiTermsUpload(self._h))

    def set_variant(self, variant: int):
        """Kernel variant (``amiSetVariant``): VARIANT_AUTO (default), VARIANT_TABLES,
        VARIANT_PACKED, VARIANT_SPECIALIZED or VARIANT_TWO_PASS (forward only)."""
        _check(load_library().amiSetVariant(self._h, int(variant)))

    def specialize(self, momentum: bool = True):
        """Compile (or load from the disk cache) and load the specialized kernels
        (``amiTermsSpecialize``) so later calls do not compile."""
        _check(load_library().amiTermsSpecialize(self._h, int(bool(momentum))))

    def source(self, momentum: bool = True, two_pass: bool = False) -> str:
        """Generated device source of the specialized kernels (``amiTermsSource``);
        ``two_pass`` for the two-pass forward's."""
        lib = load_library()
        n = ctypes.c_int64()
        sel = int(bool(momentum)) | (2 if two_pass else 0)
        _check(lib.amiTermsSource(self._h, sel, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.amiTermsSource(self._h, sel, buf, n.value, ctypes.byref(n)))
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().amiFree(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _energy_strides(energies):
    """``(tensor, stride_s, stride_i)`` of an energies tensor [N_E, nE] for the C
    ABI, whose strides must be >= 1.  A dimension of size 1 is read at index 0
    only, so its stride is irrelevant and passed as 1; a broadcast dimension
    (stride 0, e.g. ``E0.expand(N, nE)``) of size > 1 would make the kernels
    read N rows out of a buffer holding one, so such a tensor is copied to a
    contiguous one first."""
    n, m = energies.shape
    st_s, st_i = energies.stride()
    if (n > 1 and st_s < 1) or (m > 1 and st_i < 1):
        energies = energies.contiguous()
        st_s, st_i = energies.stride()
    return energies, (st_s if n > 1 else 1), (st_i if m > 1 else 1)


def _momentum_rows(k, n_int: int):
    """``(tensor, stride_k)`` of a momentum tensor [N_E, 2 n_int] (unit column
    stride) for the C ABI, which needs a row stride >= 2 n_int: rows that
    overlap or repeat (a broadcast row, stride 0) are copied to a contiguous
    tensor first; a single row's stride is irrelevant."""
    if k.shape[0] > 1 and k.stride(0) < 2 * n_int:
        k = k.contiguous()
    return k, (k.stride(0) if k.shape[0] > 1 else 2 * n_int)


def _freqs(ext_freqs, terms: Terms):
    import torch
    w = ext_freqs
    if w.dim() == 1:
        w = w.reshape(-1, 1)
    n_ext = terms.n_freq - terms.n_int
    if w.shape[1] == terms.n_freq and n_ext != terms.n_freq:
        w = w[:, terms.n_int:]          # full frequency_t rows: keep the external slots
    if w.dtype != torch.complex128 or not w.is_cuda:
        raise AmiError(-1, "ext_freqs must be a complex128 CUDA tensor")
    if w.shape[1] != n_ext:
        raise AmiError(-1, f"ext_freqs needs {n_ext} external columns")
    return w.contiguous()


def _outputs(n_f, n_e, device, want_out, want_sum, out, out_sum):
    import torch
    if want_out and out is None:
        out = torch.empty((n_f, n_e), dtype=torch.complex128, device=device)
    if want_sum and out_sum is None:
        out_sum = torch.empty((n_f,), dtype=torch.complex128, device=device)
    if out is not None and (out.dtype != torch.complex128 or tuple(out.shape) != (n_f, n_e)
                            or not out.is_contiguous() or out.device != device):
        raise AmiError(-1, f"out must be a contiguous complex128 [{n_f}, {n_e}] tensor on {device}")
    if out_sum is not None and (out_sum.dtype != torch.complex128 or tuple(out_sum.shape) != (n_f,)
                                or not out_sum.is_contiguous() or out_sum.device != device):
        raise AmiError(-1, f"out_sum must be a contiguous complex128 [{n_f}] tensor on {device}")
    return out, out_sum


def evaluate(terms: Terms, energies, ext_freqs, beta: float, e_reg: float = 0.0,
             want_out: bool = True, want_sum: bool = False, out=None, out_sum=None,
             stream=None):
    """``amiEvaluate``: energies float64 CUDA [N_E, nE] (any strides), ext_freqs
    complex128 CUDA [N_F, n_ext] (or the full [N_F, nF] rows of Sec. 2.3).
    Returns ``(out [N_F, N_E] or None, out_sum [N_F] or None)``."""
    import torch
    if energies.dtype != torch.float64 or not energies.is_cuda or energies.dim() != 2:
        raise AmiError(-1, "energies must be a 2-D float64 CUDA tensor")
    if energies.shape[1] != terms.n_eps:
        raise AmiError(-1, f"energies needs {terms.n_eps} columns")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = energies.shape[0], w.shape[0]
    out, out_sum = _outputs(n_f, n_e, energies.device, want_out, want_sum, out, out_sum)
    energies, st_s, st_i = _energy_strides(energies)
    code = load_library().amiEvaluate(
        terms._h, energies.data_ptr() if n_e else None, n_e, st_s, st_i,
        w.data_ptr(), n_f, float(beta), float(e_reg),
        out.data_ptr() if out is not None else None,
        out_sum.data_ptr() if out_sum is not None else None,
        _stream_ptr(stream))
    _check(code)
    return out, out_sum


def evaluate_complex(terms: Terms, energies, ext_freqs, beta: float, e_reg: float = 0.0,
                     want_out: bool = True, want_sum: bool = False, out=None, out_sum=None, stream=None):
    """``amiEvaluateComplex``: ``energies`` complex128 CUDA [N_E, nE] (any strides);
    returns ``(out [N_F, N_E] or None, out_sum [N_F] or None)``."""
    import torch
    if energies.dtype != torch.complex128 or not energies.is_cuda or energies.dim() != 2:
        raise AmiError(-1, "energies must be a complex128 CUDA tensor [N_E, nE]")
    if energies.shape[1] != terms.n_eps:
        raise AmiError(-1, f"energies has {energies.shape[1]} columns, terms expect {terms.n_eps}")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = energies.shape[0], w.shape[0]
    out, out_sum = _outputs(n_f, n_e, energies.device, want_out, want_sum, out, out_sum)
    energies, st_s, st_i = _energy_strides(energies)
    _check(load_library().amiEvaluateComplex(
        terms._h, energies.data_ptr() if n_e else None, n_e, st_s, st_i,
        w.data_ptr(), n_f, float(beta), float(e_reg),
        out.data_ptr() if out is not None else None,
        out_sum.data_ptr() if out_sum is not None else None, _stream_ptr(stream)))
    return out, out_sum


def evaluate_hubbard(terms: Terms, k, q: Sequence[float], t: float, mu: float, ext_freqs,
                     beta: float, e_reg: float = 0.0, want_out: bool = True,
                     want_sum: bool = False, out=None, out_sum=None, stream=None):
    """``amiEvaluateHubbard``: momenta k float64 CUDA [N_E, 2*n_int] (row-major
    rows, Sec. 5.2), external momentum q (host, 2*n_ext values), hopping t and
    chemical potential mu of eps(k) = -2t(cos kx + cos ky) - mu."""
    import torch
    if k.dtype != torch.float64 or not k.is_cuda or k.dim() != 2:
        raise AmiError(-1, "k must be a 2-D float64 CUDA tensor")
    if k.shape[1] != 2 * terms.n_int or (k.shape[0] > 0 and k.stride(1) != 1):
        raise AmiError(-1, "k must be [N_E, 2*n_int] with unit column stride")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = k.shape[0], w.shape[0]
    out, out_sum = _outputs(n_f, n_e, k.device, want_out, want_sum, out, out_sum)
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
    k, st_k = _momentum_rows(k, terms.n_int)
    code = load_library().amiEvaluateHubbard(
        terms._h, k.data_ptr() if n_e else None, n_e, st_k,
        qa.ctypes.data, float(t), float(mu), w.data_ptr(), n_f, float(beta), float(e_reg),
        out.data_ptr() if out is not None else None,
        out_sum.data_ptr() if out_sum is not None else None,
        _stream_ptr(stream))
    _check(code)
    return out, out_sum


def _ptr(t):
    return t.data_ptr() if t is not None else None


def _cot(grad_out, grad_sum, n_f, n_e, device):
    import torch
    if grad_out is not None:
        if (grad_out.dtype != torch.complex128 or tuple(grad_out.shape) != (n_f, n_e)
                or grad_out.device != device):
            raise AmiError(-1, f"grad_out must be complex128 [{n_f}, {n_e}] on {device}")
        grad_out = grad_out.contiguous()
    if grad_sum is not None:
        if grad_sum.dtype != torch.complex128 or tuple(grad_sum.shape) != (n_f,) or grad_sum.device != device:
            raise AmiError(-1, f"grad_sum must be complex128 [{n_f}] on {device}")
        grad_sum = grad_sum.contiguous()
    if grad_out is None and grad_sum is None:
        raise AmiError(-1, "grad_out and grad_sum are both None")
    return grad_out, grad_sum


def evaluate_adjoint(terms: Terms, energies, ext_freqs, beta: float, e_reg: float = 0.0,
                     grad_out=None, grad_sum=None, out=None, out_sum=None, stream=None):
    """``amiEvaluateAdjoint``: returns ``(grad_energies [N_E, nE], grad_beta [],
    grad_freqs [N_F, n_ext])`` for the cotangents of ``out`` / ``out_sum``;
    ``out`` / ``out_sum`` tensors, if given, receive the forward values."""
    import torch
    if energies.dtype != torch.float64 or not energies.is_cuda or energies.dim() != 2:
        raise AmiError(-1, "energies must be a 2-D float64 CUDA tensor")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = energies.shape[0], w.shape[0]
    dev = energies.device
    go, gs = _cot(grad_out, grad_sum, n_f, n_e, dev)
    g_e = torch.empty((n_e, terms.n_eps), dtype=torch.float64, device=dev)
    g_b = torch.empty((), dtype=torch.float64, device=dev)
    g_w = torch.empty((n_f, w.shape[1]), dtype=torch.complex128, device=dev)
    out, out_sum = _outputs(n_f, n_e, dev, False, False, out, out_sum)
    energies, st_s, st_i = _energy_strides(energies)
    _check(load_library().amiEvaluateAdjoint(
        terms._h, energies.data_ptr() if n_e else None, n_e, st_s, st_i,
        w.data_ptr(), n_f, float(beta), float(e_reg), _ptr(go), _ptr(gs),
        g_e.data_ptr() if n_e else None, g_b.data_ptr(), g_w.data_ptr(),
        _ptr(out) if n_e else None, _ptr(out_sum), _stream_ptr(stream)))
    return g_e, g_b, g_w


def evaluate_complex_adjoint(terms: Terms, energies, ext_freqs, beta: float, e_reg: float = 0.0,
                             grad_out=None, grad_sum=None, out=None, out_sum=None, stream=None):
    """``amiEvaluateComplexAdjoint``: ``energies`` complex128 CUDA [N_E, nE]
    (any strides); returns ``(grad_energies [N_E, nE] complex128 (dL/dRe E +
    i dL/dIm E), grad_beta [], grad_freqs [N_F, n_ext])`` for the cotangents of
    ``out`` / ``out_sum``; ``out`` / ``out_sum`` tensors, if given, receive the
    forward values."""
    import torch
    if energies.dtype != torch.complex128 or not energies.is_cuda or energies.dim() != 2:
        raise AmiError(-1, "energies must be a complex128 CUDA tensor [N_E, nE]")
    if energies.shape[1] != terms.n_eps:
        raise AmiError(-1, f"energies has {energies.shape[1]} columns, terms expect {terms.n_eps}")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = energies.shape[0], w.shape[0]
    dev = energies.device
    go, gs = _cot(grad_out, grad_sum, n_f, n_e, dev)
    g_e = torch.empty((n_e, terms.n_eps), dtype=torch.complex128, device=dev)
    g_b = torch.empty((), dtype=torch.float64, device=dev)
    g_w = torch.empty((n_f, w.shape[1]), dtype=torch.complex128, device=dev)
    out, out_sum = _outputs(n_f, n_e, dev, False, False, out, out_sum)
    energies, st_s, st_i = _energy_strides(energies)
    _check(load_library().amiEvaluateComplexAdjoint(
        terms._h, energies.data_ptr() if n_e else None, n_e, st_s, st_i,
        w.data_ptr(), n_f, float(beta), float(e_reg), _ptr(go), _ptr(gs),
        g_e.data_ptr() if n_e else None, g_b.data_ptr(), g_w.data_ptr(),
        _ptr(out) if n_e else None, _ptr(out_sum), _stream_ptr(stream)))
    return g_e, g_b, g_w


def evaluate_hubbard_adjoint(terms: Terms, k, q, t: float, mu: float, ext_freqs, beta: float,
                             e_reg: float = 0.0, grad_out=None, grad_sum=None, out=None,
                             out_sum=None, stream=None, grads=None):
    """``amiEvaluateHubbardAdjoint``: returns ``(grad_k [N_E, 2 n_int], grad_mu [],
    grad_t [], grad_beta [], grad_freqs [N_F, n_ext])``; ``out`` / ``out_sum``
    tensors, if given, receive the forward values.  ``grads``, if given, is a
    previous call's result whose tensors are written again instead of new ones."""
    return _hubbard_adjoint("amiEvaluateHubbardAdjoint", terms, k, q, t, mu, ext_freqs, beta, e_reg,
                            grad_out, grad_sum, out, out_sum, stream, grads)


def evaluate_hubbard_adjoint_no_alloc(terms: Terms, k, q, t: float, mu: float, ext_freqs, beta: float,
                                      e_reg: float = 0.0, grad_out=None, grad_sum=None, out=None,
                                      out_sum=None, stream=None, grads=None):
    """``amiEvaluateHubbardAdjointNoAlloc``: ``evaluate_hubbard_adjoint`` with the
    library allocating nothing (its partial sums in the library's fixed scratch).
    The handle must have been uploaded (``Terms.upload``) and, when the call runs
    specialized kernels, specialized (``Terms.specialize``) on this device.  The
    library allocates nothing; this wrapper allocates the gradient tensors unless
    ``grads`` passes a previous call's."""
    return _hubbard_adjoint("amiEvaluateHubbardAdjointNoAlloc", terms, k, q, t, mu, ext_freqs, beta, e_reg,
                            grad_out, grad_sum, out, out_sum, stream, grads)


def _hubbard_adjoint(entry: str, terms: Terms, k, q, t, mu, ext_freqs, beta, e_reg, grad_out, grad_sum,
                     out, out_sum, stream, grads):
    import torch
    if k.dtype != torch.float64 or not k.is_cuda or k.dim() != 2:
        raise AmiError(-1, "k must be a 2-D float64 CUDA tensor")
    if k.shape[1] != 2 * terms.n_int or (k.shape[0] > 0 and k.stride(1) != 1):
        raise AmiError(-1, "k must be [N_E, 2*n_int] with unit column stride")
    w = _freqs(ext_freqs, terms)
    n_e, n_f = k.shape[0], w.shape[0]
    dev = k.device
    go, gs = _cot(grad_out, grad_sum, n_f, n_e, dev)
    if grads is not None:
        g_k, g_w = grads[0], grads[4]
        scal = grads[1]._base if grads[1]._base is not None else None
        if (scal is None or tuple(scal.shape) != (3,) or tuple(g_k.shape) != (n_e, 2 * terms.n_int)
                or tuple(g_w.shape) != (n_f, w.shape[1]) or not g_k.is_contiguous()):
            raise AmiError(-1, "grads must be the result of a call of the same shape")
    else:
        g_k = torch.empty((n_e, 2 * terms.n_int), dtype=torch.float64, device=dev)
        scal = torch.empty((3,), dtype=torch.float64, device=dev)
        g_w = torch.empty((n_f, w.shape[1]), dtype=torch.complex128, device=dev)
    out, out_sum = _outputs(n_f, n_e, dev, False, False, out, out_sum)
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
    k, st_k = _momentum_rows(k, terms.n_int)
    base = scal.data_ptr()
    _check(getattr(load_library(), entry)(
        terms._h, k.data_ptr() if n_e else None, n_e, st_k,
        qa.ctypes.data, float(t), float(mu), w.data_ptr(), n_f, float(beta), float(e_reg),
        _ptr(go), _ptr(gs), g_k.data_ptr() if n_e else None, base, base + 8, base + 16,
        g_w.data_ptr(), _ptr(out) if n_e else None, _ptr(out_sum), _stream_ptr(stream)))
    return g_k, scal[0], scal[1], scal[2], g_w


def batch_source(terms_list, n_f, momentum: bool = True, compile: bool = False) -> str:
    """``amiBatchSource``: the generated source of one module of the persistent
    specialized batch for these handles (``n_f`` frequency rows each); with
    ``compile`` it is also compiled with hipRTC (no device needed)."""
    lib = load_library()
    hs = (ctypes.c_void_p * len(terms_list))(*[t._h.value for t in terms_list])
    nf = np.ascontiguousarray(np.broadcast_to(np.asarray(n_f, dtype=np.int64), (len(terms_list),)))
    n = ctypes.c_int64()
    _check(lib.amiBatchSource(hs, len(terms_list), nf.ctypes.data, int(bool(momentum)), int(bool(compile)),
                              None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib.amiBatchSource(hs, len(terms_list), nf.ctypes.data, int(bool(momentum)), 0, buf, n.value,
                              ctypes.byref(n)))
    return buf.value.decode()


def read_graph(path: str) -> np.ndarray:
    """``amiReadGraph``: the rows (source, target, B/F, spin) of a graph file, int32 [n, 4]."""
    lib = load_library()
    n = ctypes.c_int32()
    nv = ctypes.c_int32()
    _check(lib.amiReadGraph(path.encode(), None, 0, ctypes.byref(n), ctypes.byref(nv)))
    buf = np.zeros((max(n.value, 1), 4), dtype=np.int32)
    _check(lib.amiReadGraph(path.encode(), buf.ctypes.data, n.value, ctypes.byref(n), ctypes.byref(nv)))
    return buf[:n.value]


MC_MAX_FREQS = 8


def integrate_hubbard(terms: Terms, n_samples: int, seed: int, q, t: float, mu: float, ext_freqs,
                      beta: float, e_reg: float = 0.0, sums=None, stream=None):
    """``amiIntegrateHubbard``: Monte-Carlo sums over ``n_samples`` momenta drawn
    in the kernel (Philox4x32-10, ``seed``), as a float64 CUDA tensor [N_F, 4]
    of (sum Re I, sum Im I, sum (Re I)^2, sum (Im I)^2); frequency lists longer
    than 8 rows are integrated 8 rows per call (same samples for every row)."""
    import torch
    w = _freqs(ext_freqs, terms)
    n_f = w.shape[0]
    if sums is None:
        sums = torch.empty((n_f, 4), dtype=torch.float64, device=w.device)
    elif sums.dtype != torch.float64 or tuple(sums.shape) != (n_f, 4) or not sums.is_contiguous():
        raise AmiError(-1, f"sums must be contiguous float64 [{n_f}, 4]")
    qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
    lib = load_library()
    sp = _stream_ptr(stream)
    for f0 in range(0, n_f, MC_MAX_FREQS):
        f1 = min(n_f, f0 + MC_MAX_FREQS)
        _check(lib.amiIntegrateHubbard(terms._h, int(n_samples), int(seed) & 0xFFFFFFFFFFFFFFFF, qa.ctypes.data,
                                       float(t), float(mu), w[f0:f1].data_ptr(), f1 - f0, float(beta),
                                       float(e_reg), sums[f0:f1].data_ptr(), sp))
    return sums


def mc_estimate(sums, n_samples: int):
    """Mean (complex [N_F]) and standard error (float [N_F, 2], real and
    imaginary parts) of the Monte-Carlo estimate from :func:`integrate_hubbard` sums."""
    s = np.asarray(sums.cpu() if hasattr(sums, "cpu") else sums, dtype=np.float64)
    n = float(n_samples)
    mean = (s[:, 0] + 1j * s[:, 1]) / n
    var = np.stack([s[:, 2] / n - (s[:, 0] / n) ** 2, s[:, 3] / n - (s[:, 1] / n) ** 2], axis=1)
    return mean, np.sqrt(np.maximum(var, 0.0) / max(n - 1.0, 1.0))


class Batch:
    """Persistent mixed-diagram batch (``amiBatchCreate`` / ``amiBatchRun``).

    ``items`` is a list of dicts, one per diagram, each with ``terms``
    (:class:`Terms`), either ``k`` (float64 CUDA [N_E, 2 n_int], momentum path,
    with ``q``, ``t``, ``mu``) or ``energies`` (float64 CUDA [N_E, nE]),
    ``ext_freqs`` (complex128 CUDA [N_F, n_ext]), ``beta``, optional ``e_reg``,
    and the outputs ``out`` (complex128 [N_F, N_E]) and/or ``out_sum``
    (complex128 [N_F]).  The tensors are referenced by the batch; every
    :meth:`run` evaluates what they hold (an input with broadcast rows is
    copied once, here, and the batch reads the copy).  ``tuning`` is a dict with ``block``,
    ``waves_per_cu``, ``tile_factor`` and ``kernels`` (0: specialized kernels
    where AUTO would use them, as recorded launches; 1: packed only; 2: every
    item's specialized tile functions in persistent kernels; see :mod:`.autotune`).
    """

    def __init__(self, items, tuning=None):
        import torch
        lib = load_library()
        self._keep = []
        arr = (AmiBatchItem * len(items))()
        for i, it in enumerate(items):
            c = arr[i]
            t = it["terms"]
            c.terms = t.handle
            w = _freqs(it["ext_freqs"], t)
            n_f = w.shape[0]
            if "k" in it and it["k"] is not None:
                k = it["k"]
                if k.dtype != torch.float64 or not k.is_cuda or k.dim() != 2 or k.shape[1] != 2 * t.n_int \
                        or k.stride(1) != 1:
                    raise AmiError(-1, f"item {i}: k must be float64 CUDA [N_E, 2*n_int]")
                k, c.stride_k = _momentum_rows(k, t.n_int)
                c.k = k.data_ptr()
                n_e = k.shape[0]
                qa = np.asarray(it.get("q", ()), dtype=np.float64).reshape(-1)
                for j, v in enumerate(qa[:8]):
                    c.q[j] = float(v)
                c.t = float(it.get("t", 1.0))
                c.mu = float(it.get("mu", 0.0))
                self._keep.append(k)
            else:
                e = it["energies"]
                if e.dtype != torch.float64 or not e.is_cuda or e.dim() != 2 or e.shape[1] != t.n_eps:
                    raise AmiError(-1, f"item {i}: energies must be float64 CUDA [N_E, nE]")
                e, c.stride_s, c.stride_i = _energy_strides(e)
                c.energies = e.data_ptr()
                n_e = e.shape[0]
                self._keep.append(e)
            c.n_e = n_e
            c.ext_freqs = w.data_ptr()
            c.n_f = n_f
            c.beta = float(it["beta"])
            c.e_reg = float(it.get("e_reg", 0.0))
            out, out_sum = _outputs(n_f, n_e, w.device, False, False, it.get("out"), it.get("out_sum"))
            c.out = out.data_ptr() if out is not None else None
            c.out_sum = out_sum.data_ptr() if out_sum is not None else None
            self._keep += [w, out, out_sum, t]
        tun = None
        if tuning is not None:
            tun = AmiBatchTuning(int(tuning.get("block", 0)), int(tuning.get("waves_per_cu", 8)),
                                 int(tuning.get("tile_factor", 1)), int(tuning.get("kernels", 0)))
        h = ctypes.c_void_p()
        _check(lib.amiBatchCreate(arr, len(items), ctypes.byref(tun) if tun is not None else None,
                                  ctypes.byref(h)))
        self._h = h
        self.tuning = dict(tuning) if tuning is not None else None

    def run(self, stream=None):
        _check(load_library().amiBatchRun(self._h, _stream_ptr(stream)))

    def info(self) -> dict:
        buf = np.zeros(10, dtype=np.int64)
        _check(load_library().amiBatchInfo(self._h, buf.ctypes.data))
        keys = ["items", "work_items", "grid", "block", "lds_bytes", "rowsum_columns", "momentum_path",
                "lds_classes", "specialized_items", "capture_streams"]
        return {k: int(buf[i]) for i, k in enumerate(keys)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().amiBatchFree(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
