"""ctypes binding of libpdf.so: argument marshalling only.

Every computation runs in the HIP library; this module checks shapes and
dtypes, passes device pointers of PyTorch tensors, and orders the library's
stream with PyTorch's current stream.  If the library is missing the import
of a Solver fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdf.so")

PDF_OK, PDF_EINVAL, PDF_ENOMEM, PDF_EHIP, PDF_ENONFINITE, PDF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP32, FP64 = 0, 1
PARAMS_VERSION = 1
LOSS_STRIDE = 8
NKERNELS = 5
KERNEL_NAMES = ("fwd_conv", "pixel_reduce", "image_reg", "adj_gemm", "adj_conv")
LOSS_NAMES = ("state", "data", "bound", "tv", "bridge", "total", "max_abs_R", "nonfinite")

c_i32, c_f64, c_vp = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p


class Grid(ctypes.Structure):
    _fields_ = [("M", c_i32), ("side", c_f64), ("cx", c_f64), ("cy", c_f64)]


class Array(ctypes.Structure):
    _fields_ = [("n", c_i32), ("xy", ctypes.POINTER(c_f64))]


class Params(ctypes.Structure):
    _fields_ = [("version", c_i32), ("precision", c_i32),
                ("beta", c_f64), ("lam_bound", c_f64), ("lam_tv", c_f64), ("lam_bridge", c_f64),
                ("tau_b", c_f64), ("eps_tv", c_f64), ("eps_abs", c_f64),
                ("cco_tau", c_f64), ("cco_eta_max", c_f64), ("cco_delta", c_f64),
                ("gf_radius", c_i32), ("gf_eps", c_f64),
                ("lr", c_f64), ("adam_b1", c_f64), ("adam_b2", c_f64), ("adam_eps", c_f64),
                ("r_stopgrad", c_i32), ("cco_in_loss", c_i32)]


class Freq(ctypes.Structure):
    _fields_ = [("n_freq", c_i32), ("hz", ctypes.POINTER(c_f64))]


class Report(ctypes.Structure):
    _fields_ = [("iters_run", c_i32), ("n_reached", c_i32), ("seconds", c_f64)]


# name -> (restype, argtypes); every symbol declared in include/pdf.h
SIGNATURES = {
    "pdf_default_params": (c_i32, [ctypes.POINTER(Params)]),
    "pdf_setup": (c_i32, [ctypes.POINTER(Grid), c_f64, ctypes.POINTER(Array), ctypes.POINTER(Array), c_i32,
                          c_i32, ctypes.POINTER(Params), c_vp, ctypes.POINTER(c_vp)]),
    "pdf_setup_freq": (c_i32, [ctypes.POINTER(Grid), ctypes.POINTER(Freq), ctypes.POINTER(Array),
                               ctypes.POINTER(Array), c_i32, c_i32, ctypes.POINTER(Params), c_vp, ctypes.POINTER(c_vp)]),
    "pdf_tables_host": (c_i32, [ctypes.POINTER(Grid), c_f64, ctypes.POINTER(Array), ctypes.POINTER(Array),
                                c_vp, c_vp, c_vp]),
    "pdf_set_data": (c_i32, [c_vp, c_vp]),
    "pdf_loss_grad": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "pdf_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pdf_init_alpha": (c_i32, [c_vp, c_vp]),
    "pdf_init_alpha_csi": (c_i32, [c_vp, c_i32, c_vp]),
    "pdf_init_alpha_csi_noalloc": (c_i32, [c_vp, c_i32, c_vp]),
    "pdf_apply": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "pdf_mean_square": (c_i32, [c_i32, ctypes.c_int64, c_vp, c_vp, c_vp]),
    "pdf_step_multi": (c_i32, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pdf_image": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pdf_reconstruct": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                ctypes.POINTER(Report)]),
    "pdf_synthesize": (c_i32, [ctypes.POINTER(Grid), c_f64, ctypes.POINTER(Array), ctypes.POINTER(Array),
                               c_vp, c_f64, c_vp, c_vp]),
    "pdf_synthesize_batch": (c_i32, [ctypes.POINTER(Grid), c_f64, c_i32, ctypes.POINTER(Array),
                                     ctypes.POINTER(Array), c_vp, c_f64, c_vp, c_i32, c_vp, c_i32, c_vp]),
    "pdf_mlp_create": (c_i32, [c_i32, c_vp, c_i32, c_vp, ctypes.POINTER(c_vp)]),
    "pdf_mlp_set_layer": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "pdf_mlp_get_layer": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_vp]),
    "pdf_mlp_forward": (c_i32, [c_vp, c_vp, ctypes.c_float, ctypes.c_float, c_i32, c_vp]),
    "pdf_mlp_train_step": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, ctypes.c_float, c_i32, c_f64, c_vp]),
    "pdf_mlp_widths": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "pdf_mlp_destroy": (None, [c_vp]),
    "pdf_warm_start": (c_i32, [c_vp, c_vp, ctypes.c_float, ctypes.c_float, c_vp, c_vp, c_vp]),
    "pdf_analyze": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "pdf_fcnn_size": (c_i32, [c_vp, c_i32, ctypes.POINTER(ctypes.c_int64)]),
    "pdf_fcnn_forward": (c_i32, [c_vp, c_i32, c_f64, c_f64, c_vp, c_vp, c_vp]),
    "pdf_fcnn_step": (c_i32, [c_vp, c_i32, c_f64, c_f64, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]),
    "pdf_autotune": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "pdf_set_tiles": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32]),
    "pdf_reconstruct_multi": (c_i32, [c_i32, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                      c_vp]),
    "pdf_timing": (c_i32, [c_vp, c_i32, c_i32]),
    "pdf_timing_read": (c_i32, [c_vp, c_vp, c_vp]),
    "pdf_destroy": (None, [c_vp]),
    "pdf_last_error": (ctypes.c_char_p, [c_vp]),
}

_lib = None


class PdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpdf error {code}: {msg}")
        self.code = code


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_13805_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, handle=None):
    if rc != PDF_OK:
        msg = load().pdf_last_error(handle).decode()
        raise PdfError(rc, msg)


def default_params(precision: str = "fp32", **kw) -> Params:
    p = Params()
    _check(load().pdf_default_params(ctypes.byref(p)))
    p.precision = FP64 if precision == "fp64" else FP32
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _array(xy: np.ndarray):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    return Array(xy.shape[0], xy.ctypes.data_as(ctypes.POINTER(c_f64))), xy


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def tables_host(M: int, side: float, freq_hz: float, tx, rx, cx: float = 0.0, cy: float = 0.0):
    """FP64 host tables (ghat [2M,2M], gs [Ns,N], einc [Ni,N]) as computed by pdf_setup."""
    g = Grid(M, side, cx, cy)
    ta, txa = _array(tx)
    ra, rxa = _array(rx)
    ghat = np.zeros((2 * M, 2 * M), np.complex128)
    gs = np.zeros((ra.n, M * M), np.complex128)
    einc = np.zeros((ta.n, M * M), np.complex128)
    _check(load().pdf_tables_host(ctypes.byref(g), freq_hz, ctypes.byref(ta), ctypes.byref(ra),
                                  ghat.ctypes.data, gs.ctypes.data, einc.ctypes.data))
    return ghat, gs, einc


def synthesize(M: int, side: float, freq_hz: float, tx, rx, eps: np.ndarray, tol: float = 1e-10,
               device: str = "cuda:0", cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """FP64 MoM scattered field [Ni, Ns] of the permittivity map eps [M, M] (GPU)."""
    g = Grid(M, side, cx, cy)
    ta, txa = _array(tx)
    ra, rxa = _array(rx)
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.complex128))
    if eps.shape != (M, M):
        raise ValueError("eps must be [M, M]")
    out = np.zeros((ta.n, ra.n), np.complex128)
    stream = torch.cuda.Stream(device)
    torch.cuda.current_stream(device).synchronize()
    _check(load().pdf_synthesize(ctypes.byref(g), freq_hz, ctypes.byref(ta), ctypes.byref(ra),
                                 eps.ctypes.data, tol, out.ctypes.data, ctypes.c_void_p(stream.cuda_stream)))
    return out


def synthesize_batch(M: int, side: float, freq_hz: float, tx_list, rx_list, eps: np.ndarray, tol: float = 1e-10,
                     coarse: int = 0, workers: int = 0, device: str = "cuda:0", cx: float = 0.0,
                     cy: float = 0.0):
    """FP64 MoM for n instances (each with its own antenna positions) solved concurrently.

    eps: [n, M, M].  Returns E_sca [n, Ni, Ns], and with coarse = d > 0 also the
    induced currents averaged over d x d blocks, [n, Ni, M/d, M/d]."""
    g = Grid(M, side, cx, cy)
    n = len(tx_list)
    if len(rx_list) != n:
        raise ValueError("one rx array per instance is required")
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.complex128))
    if eps.shape != (n, M, M):
        raise ValueError("eps must be [n, M, M]")
    keep = [_array(t) for t in tx_list] + [_array(r) for r in rx_list]
    ta = (Array * max(n, 1))(*[k[0] for k in keep[:n]])
    ra = (Array * max(n, 1))(*[k[0] for k in keep[n:]])
    ni = len(tx_list[0]) if n else 0
    ns = len(rx_list[0]) if n else 0
    out = np.zeros((n, ni, ns), np.complex128)
    mc = M // coarse if coarse > 0 else 0
    jc = np.zeros((n, ni, mc, mc), np.complex128) if coarse > 0 else None
    stream = torch.cuda.Stream(device)
    torch.cuda.current_stream(device).synchronize()
    _check(load().pdf_synthesize_batch(ctypes.byref(g), freq_hz, n, ta, ra, eps.ctypes.data, tol, out.ctypes.data,
                                       coarse, jc.ctypes.data if jc is not None else None, workers,
                                       ctypes.c_void_p(stream.cuda_stream)))
    del keep
    return (out, jc) if coarse > 0 else out


def mean_abs2(x: torch.Tensor) -> float:
    """Mean of |x|^2 over the elements of a real or complex device tensor, computed by the
    library (pdf_mean_square); synchronous."""
    if not (isinstance(x, torch.Tensor) and x.device.type == "cuda"):
        raise ValueError("mean_abs2: expected a device tensor")
    r = torch.view_as_real(x) if x.is_complex() else x
    r = r.contiguous()
    prec = {torch.float32: FP32, torch.float64: FP64}.get(r.dtype)
    if prec is None or r.numel() < 1:
        raise ValueError("mean_abs2: expected a non-empty float32/float64 (or complex) tensor")
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    stream = torch.cuda.current_stream(x.device)
    _check(load().pdf_mean_square(prec, r.numel(), _ptr(r), _ptr(out), c_vp(stream.cuda_stream)))
    return float(out.item()) * (2.0 if x.is_complex() else 1.0)


class Solver:
    """One measurement geometry with `batch` data sets on one GPU.

    freq_hz may be a sequence of frequencies (one reconstruction, batch 1): then the
    incidence axis of alpha, the gradient and the measured fields holds the frequencies
    outermost (Ni = n_freq x antennas, [F][Ni][...] per instance)."""

    def __init__(self, M: int, side: float, freq_hz, tx, rx, K: int, batch: int = 1,
                 params: Optional[Params] = None, precision: str = "fp32", device: str = "cuda:0",
                 cx: float = 0.0, cy: float = 0.0):
        lib = load()
        self.device = torch.device(device)
        self.params = params if params is not None else default_params(precision)
        self.precision = "fp64" if self.params.precision == FP64 else "fp32"
        self.cdtype = torch.complex128 if self.precision == "fp64" else torch.complex64
        self.rdtype = torch.float64 if self.precision == "fp64" else torch.float32
        self.M, self.K, self.B = M, K, batch
        freqs = np.atleast_1d(np.asarray(freq_hz, dtype=np.float64))
        self.F = int(freqs.size)
        self.Ni, self.Ns = self.F * len(tx), len(rx)
        self.stream = torch.cuda.Stream(self.device)
        g = Grid(M, side, cx, cy)
        ta, self._tx = _array(tx)
        ra, self._rx = _array(rx)
        h = ctypes.c_void_p()
        torch.cuda.current_stream(self.device).synchronize()
        if self.F == 1:
            _check(lib.pdf_setup(ctypes.byref(g), float(freqs[0]), ctypes.byref(ta), ctypes.byref(ra), K, batch,
                                 ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h)))
        else:
            self._freqs = np.ascontiguousarray(freqs)
            fr = Freq(self.F, self._freqs.ctypes.data_as(ctypes.POINTER(c_f64)))
            _check(lib.pdf_setup_freq(ctypes.byref(g), ctypes.byref(fr), ctypes.byref(ta), ctypes.byref(ra), K,
                                      batch, ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)))
        self.h = h

    # stream ordering around each library call
    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _call(self, fn, *args):
        self._enter()
        rc = fn(self.h, *args)
        self._leave()
        _check(rc, self.h)

    def _want(self, t: torch.Tensor, shape, dtype, name, inplace: bool = False):
        """Checks device, dtype and shape.  Read-only inputs are returned
        contiguous; buffers written in place must already be contiguous."""
        ok = isinstance(t, torch.Tensor) and t.device.type == self.device.type \
            and (t.device.index or 0) == (self.device.index or 0) and t.dtype == dtype \
            and tuple(t.shape) == tuple(shape) and (t.is_contiguous() or not inplace)
        if not ok:
            got = (f"{t.dtype} {tuple(t.shape)} on {t.device}, contiguous={t.is_contiguous()}"
                   if isinstance(t, torch.Tensor) else type(t).__name__)
            raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {self.device}, got {got}")
        return t if inplace else t.contiguous()

    @property
    def alpha_shape(self):
        return (self.B, self.Ni, self.K, self.K)

    def zeros_alpha(self):
        return torch.zeros(self.alpha_shape, dtype=self.cdtype, device=self.device)

    def set_data(self, esca: torch.Tensor):
        esca = self._want(esca, (self.B, self.Ni, self.Ns), self.cdtype, "esca")
        self._call(load().pdf_set_data, _ptr(esca))

    def loss_grad(self, alpha: torch.Tensor, grad: bool = True):
        alpha = self._want(alpha, self.alpha_shape, self.cdtype, "alpha")
        loss = torch.empty((self.B, LOSS_STRIDE), dtype=torch.float64, device=self.device)
        g = torch.empty_like(alpha) if grad else None
        self._call(load().pdf_loss_grad, _ptr(alpha), _ptr(g), _ptr(loss))
        return loss, g

    def new_state(self):
        m = torch.zeros(self.alpha_shape + (2,), dtype=self.rdtype, device=self.device)
        v = torch.zeros_like(m)
        t = torch.zeros(self.B, dtype=torch.int32, device=self.device)
        return m, v, t

    def step(self, alpha, m, v, t, loss: Optional[torch.Tensor] = None):
        self._want(alpha, self.alpha_shape, self.cdtype, "alpha", inplace=True)
        self._want(m, self.alpha_shape + (2,), self.rdtype, "m", inplace=True)
        self._want(v, self.alpha_shape + (2,), self.rdtype, "v", inplace=True)
        self._want(t, (self.B,), torch.int32, "t", inplace=True)
        if loss is not None:
            self._want(loss, (self.B, LOSS_STRIDE), torch.float64, "loss", inplace=True)
        self._call(load().pdf_step, _ptr(alpha), _ptr(m), _ptr(v), _ptr(t), _ptr(loss))

    def init_alpha(self):
        a = self.zeros_alpha()
        self._call(load().pdf_init_alpha, _ptr(a))
        return a

    def fcnn_size(self, hidden: int) -> int:
        """Parameters per instance of the coefficient network with hidden width `hidden`."""
        n = ctypes.c_int64()
        _check(load().pdf_fcnn_size(self.h, hidden, ctypes.byref(n)))   # message in pdf_last_error(NULL)
        return n.value

    def fcnn_forward(self, hidden: int, alpha0: torch.Tensor, theta: torch.Tensor, s_in: float = 1.0,
                     s_out: float = 1.0):
        """alpha_hat = alpha_0 + s_out f_theta(s_in alpha_0) [B, Ni, K, K]."""
        alpha0 = self._want(alpha0, self.alpha_shape, self.cdtype, "alpha0")
        theta = self._want(theta, (self.B, self.fcnn_size(hidden)), self.rdtype, "theta")
        ah = torch.empty_like(alpha0)
        self._call(load().pdf_fcnn_forward, hidden, float(s_in), float(s_out), _ptr(alpha0), _ptr(theta), _ptr(ah))
        return ah

    def fcnn_step(self, hidden: int, alpha0: torch.Tensor, theta, m, v, t: int,
                  alpha_hat: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None,
                  s_in: float = 1.0, s_out: float = 1.0):
        """One Adam step on the network weights theta [B, n_params] in place (m, v alike, zero
        before step 1; t counts from 1).  Returns alpha_hat at the weights before the update."""
        alpha0 = self._want(alpha0, self.alpha_shape, self.cdtype, "alpha0")
        P = self.fcnn_size(hidden)
        for x, nm in ((theta, "theta"), (m, "m"), (v, "v")):
            self._want(x, (self.B, P), self.rdtype, nm, inplace=True)
        if alpha_hat is None:
            alpha_hat = torch.empty_like(alpha0)
        self._want(alpha_hat, self.alpha_shape, self.cdtype, "alpha_hat", inplace=True)
        if loss is not None:
            self._want(loss, (self.B, LOSS_STRIDE), torch.float64, "loss", inplace=True)
        self._call(load().pdf_fcnn_step, hidden, float(s_in), float(s_out), _ptr(alpha0), _ptr(theta), _ptr(m),
                   _ptr(v), int(t), _ptr(alpha_hat), _ptr(loss))
        return alpha_hat

    def init_alpha_csi(self, n_iter: int):
        """The full CSI start: n_iter conjugate-gradient steps on L^CSI (1 = init_alpha)."""
        a = self.zeros_alpha()
        self._call(load().pdf_init_alpha_csi, int(n_iter), _ptr(a))
        return a

    def init_alpha_csi_noalloc(self, n_iter: int, out: torch.Tensor):
        """init_alpha_csi into the caller's tensor `out`, with the library's static scratch as
        its workspace (the call allocates no device memory)."""
        self._want(out, self.alpha_shape, self.cdtype, "out", inplace=True)
        self._call(load().pdf_init_alpha_csi_noalloc, int(n_iter), _ptr(out))
        return out

    OPS = dict(synth=(0, "coef", "pix"), synth_adj=(1, "pix", "coef"), gd=(2, "pix", "pix"),
               gd_synth=(3, "coef", "pix"), gd_synth_adj=(4, "pix", "coef"), gs=(5, "pix", "rx"),
               gs_adj=(6, "rx", "pix"))

    def apply(self, op: str, x: torch.Tensor) -> torch.Tensor:
        """One linear piece of the loss on the whole batch: synth (B), synth_adj (B^H), gd (G_D),
        gd_synth (G_D B), gd_synth_adj (B^H G_D^H), gs (G_S), gs_adj (G_S^H)."""
        code, src, dst = self.OPS[op]
        shape = dict(coef=self.alpha_shape, pix=(self.B, self.Ni, self.M, self.M), rx=(self.B, self.Ni, self.Ns))
        x = self._want(x, shape[src], self.cdtype, "x")
        y = torch.empty(shape[dst], dtype=self.cdtype, device=self.device)
        self._call(load().pdf_apply, code, _ptr(x), _ptr(y))
        return y

    def warm_start(self, net: "Mlp", s_in: float, s_out: float):
        """Start values: the network's prediction where its loss beats the back-propagation start.

        Returns alpha [B, Ni, K, K], chosen [B] int32 (1 = network) and the two
        starts' total losses [B, 2] (back-propagation, network)."""
        a = self.zeros_alpha()
        chosen = torch.zeros(self.B, dtype=torch.int32, device=self.device)
        losses = torch.zeros((self.B, 2), dtype=torch.float64, device=self.device)
        self._call(load().pdf_warm_start, net.h, ctypes.c_float(s_in), ctypes.c_float(s_out), _ptr(a),
                   _ptr(chosen), _ptr(losses))
        return a, chosen, losses

    def analyze(self, J: torch.Tensor):
        """Kept Fourier coefficients F_T(J) [n, Ni, K, K] of pixel currents J [n, Ni, M, M]."""
        n = J.shape[0]
        J = self._want(J, (n, self.Ni, self.M, self.M), self.cdtype, "J")
        a = torch.empty((n, self.Ni, self.K, self.K), dtype=self.cdtype, device=self.device)
        self._call(load().pdf_analyze, n, _ptr(J), _ptr(a))
        return a

    def image(self, alpha, eps_true: Optional[torch.Tensor] = None):
        alpha = self._want(alpha, self.alpha_shape, self.cdtype, "alpha")
        chi = torch.empty((self.B, self.M, self.M), dtype=self.cdtype, device=self.device)
        cco = torch.empty_like(chi)
        err = None
        if eps_true is not None:
            eps_true = self._want(eps_true, (self.B, self.M, self.M), self.cdtype, "eps_true")
            err = torch.empty(self.B, dtype=torch.float64, device=self.device)
        self._call(load().pdf_image, _ptr(alpha), _ptr(chi), _ptr(cco), _ptr(eps_true), _ptr(err))
        return chi, cco, err

    def reconstruct(self, n_iter: int, n_check: int = 10, alpha: Optional[torch.Tensor] = None,
                    eps_true: Optional[torch.Tensor] = None, target: Optional[torch.Tensor] = None):
        """Start value (unless alpha is given), n_iter Adam steps from a captured
        graph, CCO image; with eps_true the image error is tracked every n_check
        steps, and with target an instance stops once its error <= target."""
        start_given = alpha is not None
        a = alpha if start_given else self.zeros_alpha()
        self._want(a, self.alpha_shape, self.cdtype, "alpha", inplace=True)
        if eps_true is not None:
            eps_true = self._want(eps_true, (self.B, self.M, self.M), self.cdtype, "eps_true")
        if target is not None:
            target = self._want(target, (self.B,), torch.float64, "target")
        track = eps_true is not None
        reached = torch.full((self.B,), -1, dtype=torch.int32, device=self.device)
        best_err = torch.empty(self.B, dtype=torch.float64, device=self.device) if track else None
        best_iter = torch.empty(self.B, dtype=torch.int32, device=self.device) if track else None
        cco = torch.empty((self.B, self.M, self.M), dtype=self.cdtype, device=self.device)
        rep = Report()
        self._call(load().pdf_reconstruct, n_iter, n_check, int(start_given), _ptr(a), _ptr(eps_true),
                   _ptr(target), _ptr(reached), _ptr(best_err), _ptr(best_iter), _ptr(cco), ctypes.byref(rep))
        return dict(alpha=a, chi_cco=cco, reached=reached, best_err=best_err, best_iter=best_iter,
                    iters_run=rep.iters_run, n_reached=rep.n_reached, seconds=rep.seconds)

    def autotune(self, reps: int = 5):
        """Times the tile and FFT-plan candidates on this handle and keeps the fastest.
        Returns ((column tiles, load batch, forward plan, adjoint plan), the nine timings in ms)."""
        choice = (c_i32 * 4)()
        ms = np.zeros(9, np.float64)
        self._call(load().pdf_autotune, reps, ctypes.cast(choice, c_vp), ms.ctypes.data)
        return tuple(choice), ms

    def set_tiles(self, ct: int, pb: int, fwd_pp: int = 0, adj_pp: int = 0):
        _check(load().pdf_set_tiles(self.h, ct, pb, fwd_pp, adj_pp), self.h)

    def timing(self, enable: bool, max_steps: int = 1000):
        """Start (or stop) recording per-kernel HIP events on the library stream."""
        _check(load().pdf_timing(self.h, int(enable), max_steps), self.h)

    def timing_read(self):
        """Average ms per kernel of the recorded iterations and their count."""
        avg = np.zeros(NKERNELS, np.float64)
        n = ctypes.c_int32()
        _check(load().pdf_timing_read(self.h, avg.ctypes.data, ctypes.byref(n)), self.h)
        return dict(zip(KERNEL_NAMES, avg.tolist())), n.value

    def close(self):
        if getattr(self, "h", None):
            load().pdf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_multi(solvers, n_iter: int, n_check: int = 10, alphas=None, eps_trues=None, targets=None):
    """Reconstructions of several solvers (any grids, antenna counts, truncations, batches) advanced
    together, one graph branch per solver.  Per-solver arguments are lists (or None); returns one
    result dict per solver as Solver.reconstruct does, and the shared step count and wall time."""
    n = len(solvers)
    if n < 1:
        raise ValueError("no solvers")
    start_given = alphas is not None
    res, keep = [], []
    arr = lambda vals: (c_vp * n)(*[None if v is None else v.data_ptr() for v in vals])
    A, E, T, RE, BE, BI, C = [], [], [], [], [], [], []
    for i, s in enumerate(solvers):
        a = alphas[i] if start_given else s.zeros_alpha()
        s._want(a, s.alpha_shape, s.cdtype, f"alphas[{i}]", inplace=True)
        et = eps_trues[i] if eps_trues is not None else None
        if et is not None:
            et = s._want(et, (s.B, s.M, s.M), s.cdtype, f"eps_trues[{i}]")
        tg = targets[i] if targets is not None else None
        if tg is not None:
            if et is None:
                raise ValueError("targets need eps_trues")
            tg = s._want(tg, (s.B,), torch.float64, f"targets[{i}]")
        track = et is not None
        r = dict(alpha=a, chi_cco=torch.empty((s.B, s.M, s.M), dtype=s.cdtype, device=s.device),
                 reached=torch.full((s.B,), -1, dtype=torch.int32, device=s.device),
                 best_err=torch.empty(s.B, dtype=torch.float64, device=s.device) if track else None,
                 best_iter=torch.empty(s.B, dtype=torch.int32, device=s.device) if track else None)
        res.append(r)
        A.append(a); E.append(et); T.append(tg); RE.append(r["reached"]); BE.append(r["best_err"])
        BI.append(r["best_iter"]); C.append(r["chi_cco"])
        s._enter()
    hs = (c_vp * n)(*[s.h.value for s in solvers])
    args = [arr(A), arr(E) if eps_trues is not None else None, arr(T) if targets is not None else None,
            arr(RE), arr(BE) if eps_trues is not None else None, arr(BI) if eps_trues is not None else None, arr(C)]
    rep = Report()
    rc = load().pdf_reconstruct_multi(n, hs, n_iter, n_check, int(start_given), *args, ctypes.byref(rep))
    for s in solvers:
        s._leave()
    _check(rc, solvers[0].h)
    for r in res:
        r.update(iters_run=rep.iters_run, seconds=rep.seconds)
    return res, dict(iters_run=rep.iters_run, n_reached=rep.n_reached, seconds=rep.seconds)


def step_multi(solvers, alphas, ms, vs, ts, losses=None):
    """One Adam step for each solver (any shapes) with its own alpha, m, v, t (and loss) tensors;
    solvers of one shape class advance in grouped launches.  Equal to separate Solver.step calls."""
    n = len(solvers)
    if n < 1 or not (len(alphas) == len(ms) == len(vs) == len(ts) == n):
        raise ValueError("one alpha, m, v and t per solver")
    for i, s in enumerate(solvers):
        s._want(alphas[i], s.alpha_shape, s.cdtype, f"alphas[{i}]", inplace=True)
        s._want(ms[i], s.alpha_shape + (2,), s.rdtype, f"ms[{i}]", inplace=True)
        s._want(vs[i], s.alpha_shape + (2,), s.rdtype, f"vs[{i}]", inplace=True)
        s._want(ts[i], (s.B,), torch.int32, f"ts[{i}]", inplace=True)
        if losses is not None:
            s._want(losses[i], (s.B, LOSS_STRIDE), torch.float64, f"losses[{i}]", inplace=True)
        s._enter()
    arr = lambda vals: (c_vp * n)(*[None if v is None else v.data_ptr() for v in vals])
    hs = (c_vp * n)(*[s.h.value for s in solvers])
    rc = load().pdf_step_multi(n, hs, arr(alphas), arr(ms), arr(vs), arr(ts),
                               arr(losses) if losses is not None else None)
    for s in solvers:
        s._leave()
    _check(rc)


class Mlp:
    """Warm-start network on one GPU: affine layers of the given widths with GELU between them.

    Weights start at zero; call init_weights or set_layer before use."""

    def __init__(self, sizes, batch_max: int, device: str = "cuda:0"):
        self.device = torch.device(device)
        self.sizes = [int(x) for x in sizes]
        self.L = len(self.sizes) - 1
        self.batch_max = int(batch_max)
        self.stream = torch.cuda.Stream(self.device)
        arr = (c_i32 * len(self.sizes))(*self.sizes)
        h = c_vp()
        torch.cuda.current_stream(self.device).synchronize()
        _check(load().pdf_mlp_create(self.L, arr, self.batch_max, c_vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def init_weights(self, seed: int):
        """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases from a seeded PCG64 stream."""
        rng = np.random.Generator(np.random.PCG64(seed))
        for l in range(self.L):
            bound = 1.0 / np.sqrt(self.sizes[l])
            W = rng.uniform(-bound, bound, size=(self.sizes[l + 1], self.sizes[l])).astype(np.float32)
            b = rng.uniform(-bound, bound, size=self.sizes[l + 1]).astype(np.float32)
            self.set_layer(l, W, b)

    def set_layer(self, l: int, W: np.ndarray, b: np.ndarray):
        W = np.ascontiguousarray(W, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        if W.shape != (self.sizes[l + 1], self.sizes[l]) or b.shape != (self.sizes[l + 1],):
            raise ValueError(f"layer {l}: expected W {(self.sizes[l + 1], self.sizes[l])} and b {(self.sizes[l + 1],)}")
        self._enter()
        _check(load().pdf_mlp_set_layer(self.h, l, W.ctypes.data, b.ctypes.data))

    def get_layer(self, l: int, grad: bool = False):
        W = np.zeros((self.sizes[l + 1], self.sizes[l]), np.float32)
        b = np.zeros(self.sizes[l + 1], np.float32)
        self._enter()
        _check(load().pdf_mlp_get_layer(self.h, l, 1 if grad else 0, W.ctypes.data, b.ctypes.data))
        return W, b

    def _rows(self, x, n, name):
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float32 and x.device == self.device
                and x.dim() == 2 and x.shape[1] == n):
            raise ValueError(f"{name}: expected float32 [rows, {n}] on {self.device}")
        return x.contiguous()

    def forward(self, x: torch.Tensor, s_in: float = 1.0, s_out: float = 1.0):
        x = self._rows(x, self.sizes[0], "x")
        B = x.shape[0]
        if not 1 <= B <= self.batch_max:
            raise ValueError(f"batch {B} outside 1..{self.batch_max}")
        y = torch.empty((B, self.sizes[-1]), dtype=torch.float32, device=self.device)
        self._enter()
        rc = load().pdf_mlp_forward(self.h, _ptr(x), ctypes.c_float(s_in), ctypes.c_float(s_out), B, _ptr(y))
        self._leave()
        _check(rc)
        return y

    def train_step(self, x: torch.Tensor, t: torch.Tensor, idx: Optional[torch.Tensor], s_in: float, lr: float,
                   loss: Optional[torch.Tensor] = None):
        """One Adam step on the MSE over rows idx of (x, t) (all rows if idx is None)."""
        x = self._rows(x, self.sizes[0], "x")
        t = self._rows(t, self.sizes[-1], "t")
        if t.shape[0] != x.shape[0]:
            raise ValueError("x and t need the same number of rows")
        if idx is not None:
            if idx.dtype != torch.int32 or idx.device != self.device or idx.dim() != 1 or idx.numel() < 1:
                raise ValueError("idx: expected int32 [B] on the network's device")
            lo, hi = int(idx.min()), int(idx.max())
            if lo < 0 or hi >= x.shape[0]:
                raise ValueError(f"idx values must lie in [0, {x.shape[0]})")
            idx = idx.contiguous()
            B = idx.shape[0]
        else:
            B = x.shape[0]
        if not 1 <= B <= self.batch_max:
            raise ValueError(f"batch {B} outside 1..{self.batch_max}")
        if loss is not None and (loss.dtype != torch.float64 or loss.numel() < 1 or not loss.is_contiguous()):
            raise ValueError("loss: expected a contiguous float64 tensor")
        self._enter()
        rc = load().pdf_mlp_train_step(self.h, _ptr(x), _ptr(t), x.shape[0], _ptr(idx), ctypes.c_float(s_in), B,
                                       float(lr), _ptr(loss))
        self._leave()
        _check(rc)

    def close(self):
        if getattr(self, "h", None):
            load().pdf_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PdfLoss(torch.autograd.Function):
    """Total PDF loss per instance with the library's hand-written adjoint.

    forward(alpha, solver, checkpoint) -> loss [B] (float64).  By default one library
    call computes loss and gradient and the gradient is kept for backward.  With
    checkpoint=True the forward runs the loss kernels only (no adjoint), alpha is kept,
    and backward runs the whole loss-gradient pass again: the adjoint's work is spent only
    when a gradient is asked for.  The saved tensor has alpha's size either way.
    """

    @staticmethod
    def forward(ctx, alpha, solver: Solver, checkpoint: bool = False):
        loss, g = solver.loss_grad(alpha.detach().contiguous(), grad=not checkpoint)
        ctx.solver = solver
        ctx.checkpoint = checkpoint
        ctx.save_for_backward(alpha.detach() if checkpoint else g)
        return loss[:, 5].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (saved,) = ctx.saved_tensors
        if ctx.checkpoint:
            _, g = ctx.solver.loss_grad(saved.contiguous(), grad=True)
        else:
            g = saved
        scale = grad_out.to(g.real.dtype).reshape(-1, 1, 1, 1)
        return g * scale, None, None
