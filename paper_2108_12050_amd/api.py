"""Python face of libmhfd: plans, detection and the soft focus score.

PyTorch provides device memory and streams; every step of the detector runs
in the HIP kernels of libmhfd, reached through the C ABI in ``_lib``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else int(t.data_ptr())


@dataclass
class Detection:
    """Blobs of one image.  ``yxk`` int32 [n, 3], ``sigma`` and ``response``
    float32 [n] (device tensors, canonical ascending (y, x, k) order);
    ``count`` is the focus criterion |C| (blobs after pruning)."""
    yxk: torch.Tensor
    sigma: torch.Tensor
    response: torch.Tensor
    count: int
    n_candidates: int
    flags: int
    stack: torch.Tensor | None = None

    @property
    def density(self) -> float:
        """Blobs per megapixel, as the library reports it (mhfd_result)."""
        return self._density

    def numpy(self):
        return (self.yxk.cpu().numpy(), self.sigma.cpu().numpy(), self.response.cpu().numpy())


def result_density(words: torch.Tensor) -> float:
    """The density field of one mhfd_result held as int64 words (host)."""
    return float(words[3:4].view(torch.float64)[0])


def split_blobs(raw: torch.Tensor, n: int):
    """View an int32 [cap, 5] buffer of mhfd_blob records as (yxk, sigma, response)."""
    r = raw[:n]
    return r[:, :3], r[:, 3].view(torch.float32), r[:, 4].view(torch.float32)


class Plan:
    """A detector configuration bound to the current device (mhfd_create_plan).

    Scales follow section 2.2's linear grid (sigma_min .. sigma_max, K = n+1
    values) unless ``sigmas`` is given.  ``threshold`` is the strict lower
    bound on the response of a candidate, ``overlap`` the pruning threshold
    (>= 1 disables pruning).  ``blur="fft"`` computes the scale space in
    the frequency domain (power-of-two tiles, radii up to 2048)."""

    def __init__(self, n_scales: int = 10, sigma_min: float = 1.0, sigma_max: float = 10.0,
                 sigmas=None, truncate: float = 4.0, threshold: float = 0.1,
                 overlap: float = 0.5, polarity: str = "bright", dtype: str = "f32",
                 max_h: int = 4096, max_w: int = 4096, max_candidates: int = 0,
                 stretch: bool = False, criterion: str = "log", sigma_cap: float | None = None,
                 blur: str = "direct"):
        self._L = _lib.load()
        self._handle = None
        cfg = _lib.Config()
        cfg.n_scales = int(n_scales if sigmas is None else len(sigmas))
        cfg.sigma_min = float(sigma_min)
        cfg.sigma_max = float(sigma_max)
        self._sig_arr = None
        if sigmas is not None:
            self._sig_arr = (C.c_float * len(sigmas))(*[float(s) for s in sigmas])
            cfg.sigmas = C.cast(self._sig_arr, C.POINTER(C.c_float))
        cfg.truncate = float(truncate)
        cfg.threshold = float(threshold)
        cfg.overlap = float(overlap)
        cfg.polarity = {"bright": _lib.MHFD_BRIGHT, "dark": _lib.MHFD_DARK}[polarity]
        cfg.in_dtype = {"f32": _lib.MHFD_F32, "u8": _lib.MHFD_U8}[dtype]
        cfg.max_h, cfg.max_w = int(max_h), int(max_w)
        cfg.max_candidates = int(max_candidates)
        cfg.stretch = 1 if stretch else 0
        cfg.criterion = {"log": _lib.MHFD_CRITERION_LOG, "dog": _lib.MHFD_CRITERION_DOG}[criterion]
        cfg.sigma_cap = 0.0 if sigma_cap is None else float(sigma_cap)
        cfg.blur = {"direct": _lib.MHFD_BLUR_DIRECT, "fft": _lib.MHFD_BLUR_FFT}[blur]
        h = C.c_void_p()
        _lib.check(self._L.mhfd_create_plan(C.byref(cfg), C.byref(h)), "mhfd_create_plan")
        self._handle = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        K = self._L.mhfd_plan_scales(h, None, None)
        sig = (C.c_float * K)()
        rad = (C.c_int32 * K)()
        self._L.mhfd_plan_scales(h, sig, rad)
        self.sigmas = [float(v) for v in sig]
        self.radii = [int(v) for v in rad]
        self.K = K
        self.dtype = dtype
        self.threshold, self.overlap, self.truncate = float(threshold), float(overlap), float(truncate)
        self.max_h, self.max_w = int(max_h), int(max_w)
        self.stretch = bool(stretch)
        self.criterion = criterion
        self.blur = blur
        # None / 0: each scale may move while its radius stays within its
        # plan radius rounded up to a multiple of 4
        self.sigma_cap = float(sigma_cap) if sigma_cap else None
        self._ws = {}
        self._focus_err = None

    def close(self):
        if self._handle is not None:
            self._L.mhfd_destroy_plan(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- workspace
    def detect_workspace_bytes(self, h: int, w: int) -> int:
        n = int(self._L.mhfd_detect_workspace_size(self._handle, int(h), int(w)))
        if n == 0:
            raise _lib.MHFDError(1, "mhfd_detect_workspace_size",
                                 f"a {h} x {w} image is empty or exceeds the plan's "
                                 f"{self.max_h} x {self.max_w}")
        return n

    def _workspace(self, key, nbytes: int) -> torch.Tensor:
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if ws.data_ptr() % 256:
                raise RuntimeError("workspace allocation not 256-byte aligned")
            self._ws[key] = ws
        return ws

    # ---------------------------------------------------------------- detect
    def detect_into(self, img: torch.Tensor, blobs_raw: torch.Tensor, result: torch.Tensor,
                    stack: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                    stream=None) -> None:
        """Enqueue mhfd_detect without synchronising.  ``blobs_raw`` is an
        int32 [capacity, 5] tensor, ``result`` an int64 [4] tensor holding
        one mhfd_result (n_blobs, n_candidates, flags, density bits)."""
        if img.dim() != 2:
            raise ValueError("image must be 2-D")
        want = torch.uint8 if self.dtype == "u8" else torch.float32
        if img.dtype != want or img.device != self.device:
            raise ValueError(f"image must be {want} on {self.device}")
        if img.stride(1) != 1:
            raise ValueError("image rows must be contiguous")
        h, w = img.shape
        if blobs_raw.dtype != torch.int32 or blobs_raw.dim() != 2 or blobs_raw.shape[1] != 5:
            raise ValueError("blobs_raw must be int32 [capacity, 5]")
        if result.dtype != torch.int64 or result.numel() < _lib.RESULT_WORDS:
            raise ValueError(f"result must be int64 [{_lib.RESULT_WORDS}]")
        if stack is not None and (stack.dtype != torch.float32 or not stack.is_contiguous()
                                  or stack.numel() != self.K * h * w):
            raise ValueError("stack must be a contiguous float32 [K, h, w] tensor")
        nbytes = self.detect_workspace_bytes(h, w)
        ws = workspace if workspace is not None else self._workspace(("detect", h, w), nbytes)
        st = self._L.mhfd_detect(self._handle, _ptr(img), h, w, img.stride(0), _ptr(blobs_raw),
                                 blobs_raw.shape[0], _ptr(result), _ptr(stack), _ptr(ws),
                                 ws.numel(), _stream_ptr(stream))
        _lib.check(st, "mhfd_detect")

    def detect(self, img: torch.Tensor, capacity: int | None = None,
               return_stack: bool = False, stream=None) -> Detection:
        """Detect blobs in one device image and wait for the result."""
        h, w = img.shape
        if capacity is None:
            capacity = max(1024, h * w // 64)
        raw = torch.empty((capacity, 5), dtype=torch.int32, device=self.device)
        res = torch.zeros(_lib.RESULT_WORDS, dtype=torch.int64, device=self.device)
        stack = (torch.empty((self.K, h, w), dtype=torch.float32, device=self.device)
                 if return_stack else None)
        self.detect_into(img, raw, res, stack, stream=stream)
        return self._finish(raw, res, capacity, h, w, stack)

    def detect_stack(self, stack: torch.Tensor, capacity: int | None = None,
                     stream=None) -> Detection:
        """The detector after the stack (mhfd_detect_stack) on a caller-held
        float32 [K, h, w] stack: window maxima, threshold, canonical list,
        pruning and count.  Waits for the result."""
        if (stack.dim() != 3 or stack.shape[0] != self.K or stack.dtype != torch.float32
                or not stack.is_contiguous() or stack.device != self.device):
            raise ValueError(f"stack must be a contiguous float32 [{self.K}, h, w] tensor on "
                             f"{self.device}")
        _, h, w = stack.shape
        if capacity is None:
            capacity = max(1024, h * w // 64)
        raw = torch.empty((capacity, 5), dtype=torch.int32, device=self.device)
        res = torch.zeros(_lib.RESULT_WORDS, dtype=torch.int64, device=self.device)
        nbytes = self.detect_workspace_bytes(h, w)
        ws = self._workspace(("detect", h, w), nbytes)
        st = self._L.mhfd_detect_stack(self._handle, _ptr(stack), h, w, _ptr(raw), capacity,
                                       _ptr(res), _ptr(ws), ws.numel(), _stream_ptr(stream))
        _lib.check(st, "mhfd_detect_stack")
        return self._finish(raw, res, capacity, h, w, stack)

    def _finish(self, raw, res, capacity, h, w, stack) -> Detection:
        host = res.cpu()
        r = host.tolist()
        n_blobs, n_cand, flags = int(r[0]), int(r[1]), int(r[2]) & 0xFFFFFFFF
        if flags & _lib.MHFD_FLAG_CAND_OVERFLOW:
            raise RuntimeError(f"{n_cand} candidates exceed the plan's candidate capacity; "
                               "create the plan with a larger max_candidates")
        n = min(n_blobs, capacity)
        yxk, sig, resp = split_blobs(raw, n)
        d = Detection(yxk, sig, resp, n_blobs, n_cand, flags, stack)
        d._density = result_density(host)
        return d

    # ---------------------------------------------------------------- soft score
    def focus_workspace_bytes(self, b: int, h: int, w: int) -> int:
        n = int(self._L.mhfd_focus_workspace_size(self._handle, int(b), int(h), int(w)))
        if n == 0:
            raise _lib.MHFDError(1, "mhfd_focus_workspace_size",
                                 f"batch {b} x {h} x {w} is empty or exceeds the plan's "
                                 f"{self.max_h} x {self.max_w}")
        return n

    def _check_soft(self, imgs: torch.Tensor, sigmas: torch.Tensor):
        if imgs.dim() == 2:
            imgs = imgs.unsqueeze(0)
        if imgs.dim() != 3 or imgs.dtype != torch.float32 or imgs.device != self.device:
            raise ValueError(f"images must be float32 [B, H, W] on {self.device}")
        if sigmas.dtype != torch.float32 or sigmas.numel() != self.K or sigmas.device != self.device:
            raise ValueError(f"sigmas must be float32 [{self.K}] on {self.device}")
        return imgs.contiguous(), sigmas.contiguous()

    def _error_word(self) -> torch.Tensor:
        if self._focus_err is None:
            self._focus_err = torch.zeros(1, dtype=torch.int32, device=self.device)
        return self._focus_err

    def check_focus_error(self, stream=None) -> None:
        """Wait for `stream` and raise if the last focus-score call on it was
        given a sigma outside (0, sigma_cap]."""
        if self._focus_err is None:
            return
        s = stream if stream is not None else torch.cuda.current_stream()
        s.synchronize()
        if int(self._focus_err.item()) & _lib.MHFD_FOCUS_BAD_SIGMA:
            allowed = (f"(0, sigma_cap = {self.sigma_cap}]" if self.sigma_cap else
                       "(0, the largest sigma whose radius fits the scale's halo]; create "
                       "the plan with sigma_cap to train further")
            raise _lib.MHFDError(1, "mhfd_focus_score", f"a sigma lies outside {allowed}")

    def focus_score(self, imgs: torch.Tensor, sigmas: torch.Tensor, beta: float = 50.0,
                    tau: float = 0.05, stream=None, check: bool = True) -> torch.Tensor:
        """S_b (float32 [B]) for device images [B, H, W].  The library reports
        a sigma outside (0, sigma_cap] in a device word; with ``check`` the
        call waits for it and raises, otherwise it returns at once and
        ``check_focus_error`` reads the word later."""
        imgs, sigmas = self._check_soft(imgs, sigmas)
        B, h, w = imgs.shape
        ws = self._workspace(("focus", B, h, w), self.focus_workspace_bytes(B, h, w))
        out = torch.empty(B, dtype=torch.float32, device=self.device)
        st = self._L.mhfd_focus_score(self._handle, _ptr(imgs), B, h, w, _ptr(sigmas),
                                      float(beta), float(tau), _ptr(out),
                                      _ptr(self._error_word()), _ptr(ws), ws.numel(),
                                      _stream_ptr(stream))
        _lib.check(st, "mhfd_focus_score")
        if check:
            self.check_focus_error(stream)
        return out

    def focus_score_backward(self, imgs: torch.Tensor, sigmas: torch.Tensor,
                             grad_scores: torch.Tensor, beta: float = 50.0, tau: float = 0.05,
                             stream=None, check: bool = True):
        """(dS/dI, dS/dsigma) contracted with grad_scores [B]; ``check`` as
        for focus_score."""
        imgs, sigmas = self._check_soft(imgs, sigmas)
        B, h, w = imgs.shape
        g = grad_scores.to(device=self.device, dtype=torch.float32).contiguous().reshape(B)
        ws = self._workspace(("focus", B, h, w), self.focus_workspace_bytes(B, h, w))
        dI = torch.empty_like(imgs)
        ds = torch.empty(self.K, dtype=torch.float32, device=self.device)
        st = self._L.mhfd_focus_score_backward(self._handle, _ptr(imgs), B, h, w, _ptr(sigmas),
                                               float(beta), float(tau), _ptr(g), _ptr(dI),
                                               _ptr(ds), _ptr(self._error_word()), _ptr(ws),
                                               ws.numel(), _stream_ptr(stream))
        _lib.check(st, "mhfd_focus_score_backward")
        if check:
            self.check_focus_error(stream)
        return dI, ds


def stretch_levels(img: torch.Tensor, stream=None):
    """Histogram stretch levels of one 8-bit device image (mhfd_stretch_levels):
    returns (levels, hist), int32 device tensors of 2 ({low, high}) and 256
    counts, enqueued on `stream` (default: the current stream)."""
    if img.dtype != torch.uint8 or img.dim() != 2 or not img.is_cuda:
        raise ValueError("stretch_levels takes a 2-D uint8 device tensor")
    if img.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    L = _lib.load()
    hist = torch.empty(256, dtype=torch.int32, device=img.device)
    levels = torch.empty(2, dtype=torch.int32, device=img.device)
    st = L.mhfd_stretch_levels(img.data_ptr(), int(img.shape[0]), int(img.shape[1]),
                               int(img.stride(0)), hist.data_ptr(), levels.data_ptr(),
                               _stream_ptr(stream))
    _lib.check(st, "mhfd_stretch_levels")
    return levels, hist


class FocusScore(torch.autograd.Function):
    """Differentiable soft focus score.  Forward and backward are the HIP
    kernels behind mhfd_focus_score / mhfd_focus_score_backward; the backward
    recomputes the per-scale responses instead of keeping a stack."""

    @staticmethod
    def forward(ctx, imgs, sigmas, plan, beta, tau):
        ctx.plan, ctx.beta, ctx.tau = plan, beta, tau
        ctx.squeeze = imgs.dim() == 2
        ctx.save_for_backward(imgs, sigmas)
        return plan.focus_score(imgs.detach(), sigmas.detach(), beta, tau)

    @staticmethod
    def backward(ctx, grad):
        imgs, sigmas = ctx.saved_tensors
        dI, ds = ctx.plan.focus_score_backward(imgs.detach(), sigmas.detach(), grad, ctx.beta,
                                               ctx.tau)
        if ctx.squeeze:
            dI = dI[0]
        return (dI if ctx.needs_input_grad[0] else None,
                ds if ctx.needs_input_grad[1] else None, None, None, None)


def focus_score(imgs: torch.Tensor, sigmas: torch.Tensor, plan: Plan, beta: float = 50.0,
                tau: float = 0.05) -> torch.Tensor:
    """S_b = mean over scales and pixels of softplus(beta (|sigma^2 Lap(G_sigma * I)| - tau)),
    differentiable in the images and the sigmas; each call takes every
    scale's radius floor(truncate sigma + 0.5) from the current sigma and
    raises if a sigma leaves (0, plan.sigma_cap]."""
    return FocusScore.apply(imgs, sigmas, plan, float(beta), float(tau))
