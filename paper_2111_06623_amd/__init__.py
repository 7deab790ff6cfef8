"""Python binding of the lz C ABI (include/lz.h): argument marshalling only.

Every computation runs in the HIP library liblz.so (built for gfx950 by
``paper_2111_06623_amd.build``).  Importing this package never computes
anything; ``load()`` raises if the library is missing rather than falling back
to any other implementation.

Device vectors are torch tensors on the GPU (complex128 for LZ_FP64,
complex64 for the mixed modes), shaped [nks, nbnd, npwx] per instance and
concatenated over instances; torch supplies memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LZ_OK, LZ_ERR_ARG, LZ_ERR_HIP, LZ_ERR_OOM, LZ_ERR_NOT_PD, LZ_ERR_STATE, LZ_BREAKDOWN = range(7)
LZ_FP64, LZ_FP32, LZ_FP32_SPLITBF16 = 0, 1, 2
LZ_TDDFT, LZ_RPA, LZ_IPA = 0, 1, 2
APPROX = {"tddft": LZ_TDDFT, "rpa": LZ_RPA, "ipa": LZ_IPA}
PREC = {"fp64": LZ_FP64, "fp32": LZ_FP32, "splitbf16": LZ_FP32_SPLITBF16}
LZ_EXTRAP_NONE, LZ_EXTRAP_CONSTANT, LZ_EXTRAP_OSC = 0, 1, 2
EXTRAPOLATION = {"no": LZ_EXTRAP_NONE, "constant": LZ_EXTRAP_CONSTANT, "osc": LZ_EXTRAP_OSC}
LZ_PSEUDO_HERMITIAN, LZ_NON_HERMITIAN = 0, 1
ALGORITHM = {"ph": LZ_PSEUDO_HERMITIAN, "nh": LZ_NON_HERMITIAN}
LZ_GEMM_AUTO, LZ_GEMM_VALU, LZ_GEMM_MFMA = 0, 1, 2
GEMM = {"auto": LZ_GEMM_AUTO, "valu": LZ_GEMM_VALU, "mfma": LZ_GEMM_MFMA}
FFT_PLANES = {"auto": 0, "registers": 1, "lds": 2}
STATUS_NAMES = {0: "ok", 1: "arg", 2: "hip", 3: "oom", 4: "not_pd", 5: "state", 6: "breakdown"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblz.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class LzSystem(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int32 * 3), ("at", ctypes.c_double * 9), ("q", ctypes.c_double * 3),
        ("g0", ctypes.c_int32 * 3),
        ("nks", ctypes.c_int32), ("nbnd", ctypes.c_int32), ("nproj", ctypes.c_int32),
        ("npwx", ctypes.c_int32),
        ("xk", _dp), ("wk", _dp), ("npw_k", _ip), ("npw_kq", _ip), ("nl_k", _ip), ("nl_kq", _ip),
        ("evc_k", _dp), ("evc_kq", _dp), ("et_k", _dp), ("vloc_r", _dp), ("fxc_r", _dp),
        ("vkb_kq", _dp), ("dkb", _dp),
    ]


class LzOptions(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("approx", ctypes.c_int), ("max_steps", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("algorithm", ctypes.c_int), ("streams", ctypes.c_int32),
                ("projector_gemm", ctypes.c_int), ("density_group_bands", ctypes.c_int32),
                ("projector_chunk", ctypes.c_int32), ("fft_planes", ctypes.c_int32),
                ("batched", ctypes.c_int32)]


class LzError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lz status {status} ({STATUS_NAMES.get(status, '?')}): {msg}")
        self.status = status


STAGES = ["zfft_inv", "plane_local", "plane_density", "hxc", "plane_vu", "zfft_fwd",
          "projectors", "lanczos"]


def load(path: str = LIB_PATH):
    """Load liblz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_2111_06623_amd.build")
    # torch first: it carries its own HIP runtime under the same soname, and
    # the library must bind to the runtime that owns torch's streams and
    # memory (loaded the other way round, the process holds two runtimes and
    # device discovery fails)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.lz_init.argtypes = [ctypes.POINTER(LzSystem), ctypes.c_int32, ctypes.POINTER(LzOptions),
                            ctypes.c_int32, vp, ctypes.POINTER(vp)]
    lib.lz_apply_liouvillian.argtypes = [vp, vp, vp, vp, vp]
    lib.lz_step.argtypes = [vp, ctypes.c_int32, _ip]
    lib.lz_get_coefficients.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp]
    lib.lz_get_state.argtypes = [vp, ctypes.c_int32, _ip, _ip]
    lib.lz_get_gamma.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp]
    lib.lz_get_tuning.argtypes = [vp, ctypes.c_int32, _ip, _ip, _ip, _ip]
    lib.lz_ground_state.argtypes = [ctypes.POINTER(LzSystem), ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_int32, vp, _dp, _dp, _ip, _dp]
    lib.lz_ground_density.argtypes = [ctypes.POINTER(LzSystem), ctypes.c_int32, ctypes.c_int32, vp,
                                      _dp, _dp]
    lib.lz_spectrum.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_int32,
                                ctypes.c_double, _dp, _dp, _dp]
    lib.lz_spectrum_ext.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    _dp, ctypes.c_int32, ctypes.c_double, _dp, _dp, _dp]
    lib.lz_spectrum_ext_noalloc.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, _dp, ctypes.c_int32, ctypes.c_double,
                                            _dp, _dp, _dp]
    lib.lz_checkpoint_size.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
    lib.lz_checkpoint_save.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_uint64]
    lib.lz_checkpoint_load.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_uint64]
    lib.lz_get_rhs.argtypes = [vp, ctypes.c_int32, vp]
    lib.lz_reset.argtypes = [vp]
    lib.lz_stage_timer.argtypes = [vp, ctypes.c_int32]
    lib.lz_stage_times.argtypes = [vp, ctypes.c_int32, _dp, _ip]
    lib.lz_free.argtypes = [vp]
    lib.lz_launch_plan.argtypes = [ctypes.c_int32] * 7 + [_ip]
    lib.lz_last_error.restype = ctypes.c_char_p
    for f in ("lz_init", "lz_apply_liouvillian", "lz_step", "lz_get_coefficients", "lz_get_gamma",
              "lz_get_tuning", "lz_ground_state", "lz_ground_density",
              "lz_get_state",
              "lz_spectrum", "lz_spectrum_ext", "lz_spectrum_ext_noalloc", "lz_checkpoint_size", "lz_checkpoint_save",
              "lz_checkpoint_load", "lz_get_rhs", "lz_reset", "lz_stage_timer", "lz_stage_times", "lz_free"):
        getattr(lib, f).restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def lz_last_error() -> str:
    return load().lz_last_error().decode()


def _check(status, allow=()):
    if status != LZ_OK and status not in allow:
        raise LzError(status, lz_last_error())
    return status


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def make_system(s):
    """Marshal a system (any object with the lz_system fields as arrays) into
    an LzSystem; returns (struct, keepalive)."""
    keep = dict(
        xk=_f64(s.xk), wk=_f64(s.wk), npw_k=_i32(s.npw_k), npw_kq=_i32(s.npw_kq),
        nl_k=_i32(s.nl_k), nl_kq=_i32(s.nl_kq), evc_k=_c128(s.evc_k), evc_kq=_c128(s.evc_kq),
        et_k=_f64(s.et_k), vloc_r=_f64(s.vloc_r), fxc_r=_f64(s.fxc_r),
        vkb_kq=_c128(s.vkb_kq) if len(s.dkb) else None, dkb=_f64(s.dkb) if len(s.dkb) else None)
    st = LzSystem()
    st.nr[:] = [int(v) for v in s.nr]
    st.at[:] = [float(v) for v in np.asarray(s.at, dtype=np.float64).ravel()]
    st.q[:] = [float(v) for v in s.q]
    st.g0[:] = [int(v) for v in s.g0]
    st.nks = int(np.asarray(s.xk).shape[0])
    st.nbnd = int(np.asarray(s.et_k).shape[1])
    st.nproj = int(len(s.dkb))
    st.npwx = int(np.asarray(s.nl_kq).shape[1])
    for name in ("xk", "wk", "evc_k", "evc_kq", "et_k", "vloc_r", "fxc_r", "vkb_kq", "dkb"):
        setattr(st, name, _ptr(keep[name], _dp))
    for name in ("npw_k", "npw_kq", "nl_k", "nl_kq"):
        setattr(st, name, _ptr(keep[name], _ip))
    return st, keep


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def lz_init(systems, prec="fp64", approx="tddft", max_steps=1000, use_graph=False, autotune=False,
            device=0, stream=None, algorithm="ph", streams=0, projector_gemm="auto",
            density_group_bands=0, projector_chunk=0, fft_planes="auto", batched=False):
    """Create a context for one system or a list of systems; returns a handle.
    algorithm: "ph" (pseudo-Hermitian) or "nh" (non-Hermitian biorthogonal);
    streams: instances stepped side by side (0: the library default);
    batched: lz_step runs one launch per kernel over all instances (work list);
    projector_gemm: "auto", "valu" or "mfma" (where the projector products run);
    density_group_bands, projector_chunk: fixed launch parameters (0: heuristic
    or autotuned); fft_planes: "auto", "registers" (register-line / lane-pair
    plane transforms where they exist) or "lds" (LDS Stockham passes)."""
    lib = load()
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    arr = (LzSystem * len(systems))()
    keep = []
    for i, s in enumerate(systems):
        arr[i], k = make_system(s)
        keep.append(k)
    opt = LzOptions(PREC[prec] if isinstance(prec, str) else int(prec),
                    APPROX[approx] if isinstance(approx, str) else int(approx),
                    int(max_steps), int(bool(use_graph)), int(bool(autotune)),
                    ALGORITHM[algorithm] if isinstance(algorithm, str) else int(algorithm),
                    int(streams),
                    GEMM[projector_gemm] if isinstance(projector_gemm, str) else int(projector_gemm),
                    int(density_group_bands), int(projector_chunk),
                    FFT_PLANES[fft_planes] if isinstance(fft_planes, str) else int(fft_planes),
                    int(bool(batched)))
    out = ctypes.c_void_p()
    hs = _stream_handle(device) if stream is None else ctypes.c_void_p(stream)
    _check(lib.lz_init(arr, len(systems), ctypes.byref(opt), int(device), hs, ctypes.byref(out)))
    return Context(out, systems, opt)


def lz_ground_state(system, nbnd=None, n_extra=4, tol=1e-9, max_iter=300, device=0, stream=None):
    """The lowest nbnd eigenpairs of H_{k+q} on every k+q sphere of `system`
    (lz_ground_state).  Returns (evc [nks][nbnd][npwx] complex128 in the
    order of nl_kq, eps [nks][nbnd], iterations, max residual norm)."""
    import copy
    lib = load()
    s = copy.copy(system)
    nb = int(np.asarray(s.et_k).shape[1]) if nbnd is None else int(nbnd)
    nks = int(np.asarray(s.xk).shape[0])
    npwx = int(np.asarray(s.nl_kq).shape[1])
    # placeholders of the right shapes for the fields the solver does not read
    s.evc_k = np.zeros((nks, nb, npwx), dtype=np.complex128)
    s.evc_kq = s.evc_k
    s.et_k = np.zeros((nks, nb))
    if getattr(s, "fxc_r", None) is None:
        s.fxc_r = np.zeros_like(np.asarray(s.vloc_r))
    arr, keep = make_system(s)
    evc = np.zeros(nks * nb * npwx * 2)
    eps = np.zeros(nks * nb)
    it = ctypes.c_int32()
    res = ctypes.c_double()
    hs = _stream_handle(device) if stream is None else ctypes.c_void_p(stream)
    _check(lib.lz_ground_state(ctypes.byref(arr), int(n_extra), float(tol), int(max_iter),
                               int(device), hs, _ptr(evc, _dp), _ptr(eps, _dp), ctypes.byref(it),
                               ctypes.byref(res)))
    return (evc.view(np.complex128).reshape(nks, nb, npwx), eps.reshape(nks, nb), int(it.value),
            float(res.value))


XC = {"x": 0, "pz": 1}


def lz_ground_density(system, xc="pz", device=0, stream=None):
    """Ground-state density n0 and the LDA kernel f_xc(n0) from the orbitals
    at k of `system` (lz_ground_density); returns (n0, fxc), grid order of
    vloc_r."""
    import copy
    lib = load()
    s = copy.copy(system)
    nks, nb = (int(v) for v in np.asarray(s.evc_k).shape[:2])
    # placeholders of the right shapes for the fields the call does not read
    s.evc_kq = s.evc_k
    s.et_k = np.zeros((nks, nb))
    s.fxc_r = np.zeros_like(np.asarray(s.vloc_r))
    arr, keep = make_system(s)
    N = int(np.prod(np.asarray(s.nr)))
    n0 = np.zeros(N)
    fxc = np.zeros(N)
    hs = _stream_handle(device) if stream is None else ctypes.c_void_p(stream)
    _check(lib.lz_ground_density(ctypes.byref(arr), XC[xc] if isinstance(xc, str) else int(xc),
                                 int(device), hs, _ptr(n0, _dp), _ptr(fxc, _dp)))
    return n0, fxc


LZ_PLAN_LEN = 15
PLAN_FIELDS = ("ct_size", "reg_plane", "group_reg", "group_lds", "group_round",
               "valu_chunk", "valu_nchunk", "valu_upd_blocks", "valu_upd_blocks_proj",
               "mfma_chunk", "mfma_nchunk", "mfma_upd_blocks", "mfma_upd_blocks_proj",
               "gsize", "ngroups")


def lz_launch_plan(n, prec, nbnd, nks, npwx, nproj, slots=0):
    """Host-side launch plan of a cubic grid (lz_launch_plan; no device):
    a dict of the LZ_PLAN_LEN fields named in PLAN_FIELDS."""
    lib = load()
    out = np.zeros(LZ_PLAN_LEN, dtype=np.int32)
    _check(lib.lz_launch_plan(int(n), PREC[prec] if isinstance(prec, str) else int(prec),
                              int(nbnd), int(nks), int(npwx), int(nproj), int(slots),
                              _ptr(out, _ip)))
    return dict(zip(PLAN_FIELDS, (int(v) for v in out)))


class Context:
    """Handle of an lz context; methods call the C ABI of the same name."""

    def __init__(self, handle, systems, opt):
        self.handle = handle
        self.prec = opt.prec
        self.algorithm = opt.algorithm
        self.nvec = [int(np.asarray(s.xk).shape[0]) * int(np.asarray(s.et_k).shape[1]) *
                     int(np.asarray(s.nl_kq).shape[1]) for s in systems]
        self.shapes = [(int(np.asarray(s.xk).shape[0]), int(np.asarray(s.et_k).shape[1]),
                        int(np.asarray(s.nl_kq).shape[1])) for s in systems]

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.prec == LZ_FP64 else torch.complex64

    def _dev(self, t):
        if t is None:
            return None
        if not t.is_cuda or not t.is_contiguous() or t.dtype != self.complex_dtype or t.numel() != sum(self.nvec):
            raise ValueError("vectors must be contiguous CUDA tensors of the context's dtype and size")
        return ctypes.c_void_p(t.data_ptr())

    def apply_liouvillian(self, q_in, p_in, q_out, p_out):
        lib = load()
        _check(lib.lz_apply_liouvillian(self.handle, self._dev(q_in), self._dev(p_in),
                                        self._dev(q_out), self._dev(p_out)))

    def step(self, n):
        lib = load()
        done = ctypes.c_int32()
        st = _check(lib.lz_step(self.handle, int(n), ctypes.byref(done)), allow=(LZ_BREAKDOWN,))
        return int(done.value), st

    def reset(self):
        """Restart the recursion from (0, y) (lz_reset)."""
        _check(load().lz_reset(self.handle))

    def state(self, inst=0):
        lib = load()
        n, st = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.lz_get_state(self.handle, int(inst), ctypes.byref(n), ctypes.byref(st)))
        return int(n.value), int(st.value)

    def coefficients(self, inst=0, first=0, count=None):
        lib = load()
        if count is None:
            count = self.state(inst)[0] - first
        beta = np.zeros(count)
        gamma = np.zeros(2 * count)
        z = np.zeros(2 * count)
        _check(lib.lz_get_coefficients(self.handle, int(inst), int(first), int(count),
                                       _ptr(beta, _dp), None, _ptr(z, _dp)))
        _check(lib.lz_get_gamma(self.handle, int(inst), int(first), int(count), _ptr(gamma, _dp)))
        gamma = gamma.view(np.complex128)
        if self.algorithm == LZ_PSEUDO_HERMITIAN:
            gamma = gamma.real.copy()
        return beta, gamma, z.view(np.complex128)

    def spectrum(self, omega, eta, m=None, inst=0, m_total=None, extrapolation="no"):
        """chi, eps^-1 and the loss function from the first m coefficients
        (default: all computed), with extrapolation 'constant' or 'osc' of the
        tridiagonal matrix to dimension m_total (lz_spectrum_ext)."""
        lib = load()
        omega = _f64(omega)
        if m is None:
            m = self.state(inst)[0]
        scheme = EXTRAPOLATION[extrapolation] if isinstance(extrapolation, str) else int(extrapolation)
        mt = int(m if m_total is None else m_total)
        chi = np.zeros(2 * len(omega))
        einv = np.zeros(2 * len(omega))
        loss = np.zeros(len(omega))
        _check(lib.lz_spectrum_ext(self.handle, int(inst), int(m), mt, scheme, _ptr(omega, _dp),
                                   len(omega), float(eta), _ptr(chi, _dp), _ptr(einv, _dp),
                                   _ptr(loss, _dp)))
        return chi.view(np.complex128), einv.view(np.complex128), loss

    def spectrum_noalloc(self, omega, eta, m=None, inst=0, m_total=None, extrapolation="no"):
        """As spectrum(), through lz_spectrum_ext_noalloc (no device allocation;
        at most 65536 frequencies)."""
        lib = load()
        omega = _f64(omega)
        if m is None:
            m = self.state(inst)[0]
        scheme = EXTRAPOLATION[extrapolation] if isinstance(extrapolation, str) else int(extrapolation)
        mt = int(m if m_total is None else m_total)
        chi = np.zeros(2 * len(omega))
        einv = np.zeros(2 * len(omega))
        loss = np.zeros(len(omega))
        _check(lib.lz_spectrum_ext_noalloc(self.handle, int(inst), int(m), mt, scheme,
                                           _ptr(omega, _dp), len(omega), float(eta),
                                           _ptr(chi, _dp), _ptr(einv, _dp), _ptr(loss, _dp)))
        return chi.view(np.complex128), einv.view(np.complex128), loss

    def tuning(self, inst=0):
        """(projector path name, density band-group size, projector dot chunks,
        plane-transform schedule "registers" or "lds") of one instance
        (lz_get_tuning)."""
        g, b, c, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().lz_get_tuning(self.handle, int(inst), ctypes.byref(g), ctypes.byref(b),
                                    ctypes.byref(c), ctypes.byref(f)))
        return ({LZ_GEMM_VALU: "valu", LZ_GEMM_MFMA: "mfma"}[g.value], int(b.value), int(c.value),
                {1: "registers", 2: "lds"}[f.value])

    def checkpoint(self, inst=0):
        """The recursion state of one instance as bytes (lz_checkpoint_save)."""
        lib = load()
        n = ctypes.c_uint64()
        _check(lib.lz_checkpoint_size(self.handle, int(inst), ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.lz_checkpoint_save(self.handle, int(inst), buf, n.value))
        return buf.raw

    def restore(self, blob, inst=0):
        """Continue from a checkpoint of the same system (lz_checkpoint_load)."""
        lib = load()
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(lib.lz_checkpoint_load(self.handle, int(inst), buf, len(blob)))

    def rhs(self, inst=0):
        import torch
        lib = load()
        y = torch.zeros(self.shapes[inst], dtype=self.complex_dtype, device="cuda")
        _check(lib.lz_get_rhs(self.handle, int(inst), ctypes.c_void_p(y.data_ptr())))
        return y

    def stage_timer(self, enable=True, stages=None):
        """Time every stage (enable), none, or only the stages named in
        `stages` (names from STAGES) with HIP events (lz_stage_timer)."""
        mask = 0
        if enable:
            mask = -1 if stages is None else sum(1 << STAGES.index(n) for n in stages)
        _check(load().lz_stage_timer(self.handle, int(mask)))

    def stage_times(self, inst=0):
        """(total_ms[8], count[8]) per stage since the last stage_timer call."""
        ms = np.zeros(8)
        cnt = np.zeros(8, dtype=np.int32)
        _check(load().lz_stage_times(self.handle, int(inst), _ptr(ms, _dp), _ptr(cnt, _ip)))
        return ms, cnt

    def free(self):
        if self.handle:
            load().lz_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# functional aliases with the C names
def lz_apply_liouvillian(ctx, q_in, p_in, q_out, p_out):
    return ctx.apply_liouvillian(q_in, p_in, q_out, p_out)


def lz_step(ctx, n):
    return ctx.step(n)


def lz_get_coefficients(ctx, inst=0, first=0, count=None):
    return ctx.coefficients(inst, first, count)


def lz_reset(ctx):
    return ctx.reset()


def lz_get_state(ctx, inst=0):
    return ctx.state(inst)


def lz_spectrum(ctx, omega, eta, m=None, inst=0):
    return ctx.spectrum(omega, eta, m, inst)


def lz_get_rhs(ctx, inst=0):
    return ctx.rhs(inst)


def lz_free(ctx):
    ctx.free()
