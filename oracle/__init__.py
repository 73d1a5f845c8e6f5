"""FP64 CPU oracle for the MHFD scale-normalised LoG blob detector.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The C file
``mhfd_oracle.c`` beside this one holds the arithmetic; this module builds it
with gcc, loads it with ctypes and converts arrays.  Nothing here shares code
with the HIP path.

Paper anchors (arXiv 2108.12050):
  * Gaussian, scale space, std-as-scale: section 2.2.
  * Scale-normalised Laplacian (t^2 Lap L): section 2.2, equation
    "blobdetector" and the DoG approximation after it.
  * Scale grid n, min_t, max_t, delta t, t_i: section 2.2.
  * Feature set C as maxpool-equality maxima and its cardinality |C| as the
    criterion: section 3, equation "argmax", and Algorithm 1 (Ensure).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhfd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmhfd_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_bp = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, IEEE double)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.ora_radius.restype = C.c_int
        L.ora_radius.argtypes = [C.c_double, C.c_double]
        L.ora_taps.argtypes = [C.c_double, C.c_int, _dp, _dp]
        L.ora_dtaps.argtypes = [C.c_double, C.c_int, _dp, _dp]
        L.ora_ext.restype = C.c_long
        L.ora_ext.argtypes = [C.c_long, C.c_long]
        L.ora_log_stack.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_int, _dp]
        L.ora_log_direct.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_int, _dp]
        L.ora_log_point.restype = C.c_double
        L.ora_log_point.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                    C.c_int, C.c_int]
        L.ora_candidates.restype = C.c_long
        L.ora_candidates.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, _ip, _dp, C.c_long]
        L.ora_ambiguous.restype = C.c_long
        L.ora_ambiguous.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_void_p]
        L.ora_overlap.restype = C.c_double
        L.ora_overlap.argtypes = [C.c_double] * 6
        L.ora_prune.argtypes = [_ip, _dp, C.c_long, C.c_double, _bp]
        L.ora_soft_score.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _ip,
                                     C.c_double, C.c_double, _dp]
        L.ora_soft_score_grad.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _ip,
                                          C.c_double, C.c_double, _dp, _dp, _dp]
        L.ora_log_adjoint.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _dp]
        _u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        _i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        _intp = C.POINTER(C.c_int)
        L.ora_stretch_levels.argtypes = [_u8p, C.c_int, C.c_int, C.c_long, _i64p, _intp, _intp]
        L.ora_stretch.argtypes = [_u8p, C.c_int, C.c_int, C.c_long, _dp, _intp, _intp]
        L.ora_gauss_stack.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, _dp]
        _i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.ora_dog_criterion.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, _dp,
                                        _i32p, _i32p, C.c_long]
        L.ora_dog_criterion.restype = C.c_long
        L.ora_threads.restype = C.c_int
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_set_threads.restype = None
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().ora_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's parallel loops from now on (timing only)."""
    lib().ora_set_threads(int(n))


# ----------------------------------------------------------------------------
# inputs
# ----------------------------------------------------------------------------

def to_f64(img) -> np.ndarray:
    """Image as FP64: fp32 values exactly, or u/255 for 8-bit input."""
    a = np.asarray(img)
    if a.dtype == np.uint8:
        return np.ascontiguousarray(a.astype(np.float64) / 255.0)
    return np.ascontiguousarray(a.astype(np.float64))


def linear_sigmas(K: int, smin: float, smax: float) -> np.ndarray:
    """Scale grid of section 2.2: t_i = min_t + (i-1) delta_t for K = n+1
    scales, delta_t = (max_t - min_t)/n; each value is rounded to FP32 (the
    precision the detector's configuration holds) and returned as FP64."""
    if K == 1:
        vals = [smin]
    else:
        dt = (smax - smin) / (K - 1)
        vals = [smin + i * dt for i in range(K)]
    return np.asarray(np.float32(vals), dtype=np.float64)


# ----------------------------------------------------------------------------
# taps and border extension
# ----------------------------------------------------------------------------

def radius(sigma: float, truncate: float = 4.0) -> int:
    return int(lib().ora_radius(float(sigma), float(truncate)))


def taps(sigma: float, R: int):
    g = np.zeros(2 * R + 1)
    h = np.zeros(2 * R + 1)
    lib().ora_taps(float(sigma), int(R), g, h)
    return g, h


def dtaps(sigma: float, R: int):
    gd = np.zeros(2 * R + 1)
    hd = np.zeros(2 * R + 1)
    lib().ora_dtaps(float(sigma), int(R), gd, hd)
    return gd, hd


def ext(u: int, n: int) -> int:
    return int(lib().ora_ext(int(u), int(n)))


# ----------------------------------------------------------------------------
# LoG stack
# ----------------------------------------------------------------------------

def log_stack(img, sigmas, truncate: float = 4.0, polarity: int = 0) -> np.ndarray:
    """K x H x W stack of s * sigma_k^2 * Lap(G_sigma_k * I) (separable form)."""
    I = to_f64(img)
    H, W = I.shape
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    out = np.zeros((len(sg), H, W))
    lib().ora_log_stack(I, H, W, len(sg), sg, float(truncate), int(polarity), out)
    return out


def log_direct(img, sigmas, truncate: float = 4.0, polarity: int = 0) -> np.ndarray:
    """Same stack from the plain 2-D square-support sum (tiny images only)."""
    I = to_f64(img)
    H, W = I.shape
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    out = np.zeros((len(sg), H, W))
    lib().ora_log_direct(I, H, W, len(sg), sg, float(truncate), int(polarity), out)
    return out


def log_point(img, sigma: float, y: int, x: int, truncate: float = 4.0,
              polarity: int = 0) -> float:
    """One voxel from the 2-D definition; `img` must already be FP64."""
    I = img if (isinstance(img, np.ndarray) and img.dtype == np.float64
                and img.flags.c_contiguous) else to_f64(img)
    H, W = I.shape
    return float(lib().ora_log_point(I, H, W, float(sigma), float(truncate), int(polarity),
                                     int(y), int(x)))


def log_adjoint(c, sigma: float, truncate: float = 4.0, polarity: int = 0) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    H, W = c.shape
    out = np.zeros((H, W))
    lib().ora_log_adjoint(c, H, W, float(sigma), float(truncate), int(polarity), out)
    return out


# ----------------------------------------------------------------------------
# detection
# ----------------------------------------------------------------------------

def candidates(stack: np.ndarray, tau: float):
    """3x3x3 window maxima above tau, ascending (y, x, k)."""
    st = np.ascontiguousarray(stack, dtype=np.float64)
    K, H, W = st.shape
    cap = 1 << 16
    while True:
        ykx = np.zeros((cap, 3), dtype=np.int32)
        resp = np.zeros(cap)
        n = int(lib().ora_candidates(st, K, H, W, float(tau), ykx, resp, cap))
        if n <= cap:
            return ykx[:n].copy(), resp[:n].copy()
        cap = n


def ambiguous(stack: np.ndarray, tau: float, eps: float, mask: bool = False):
    """Number of voxels whose candidate decision is within eps of flipping
    (and the K x H x W mask of them when `mask`)."""
    st = np.ascontiguousarray(stack, dtype=np.float64)
    K, H, W = st.shape
    if mask:
        m = np.zeros((K, H, W), dtype=np.uint8)
        n = int(lib().ora_ambiguous(st, K, H, W, float(tau), float(eps),
                                    m.ctypes.data_as(C.c_void_p)))
        return n, m.astype(bool)
    return int(lib().ora_ambiguous(st, K, H, W, float(tau), float(eps), None))


def overlap(ya, xa, ra, yb, xb, rb) -> float:
    return float(lib().ora_overlap(float(ya), float(xa), float(ra),
                                   float(yb), float(xb), float(rb)))


def prune(ykx, sigmas, theta: float) -> np.ndarray:
    """Keep mask of the one-shot dominance prune (True = kept)."""
    ykx = np.ascontiguousarray(np.asarray(ykx, dtype=np.int32).reshape(-1, 3))
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    keep = np.zeros(len(ykx), dtype=np.uint8)
    if len(ykx):
        lib().ora_prune(ykx, sg, len(ykx), float(theta), keep)
    return keep.astype(bool)


def stretch_levels(img: np.ndarray):
    """(low, high, hist) of the histogram stretch of an 8-bit image (section 3,
    Algorithm 1 first step; 0.175% saturated at each end)."""
    a = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = a.shape
    hist = np.zeros(256, np.int64)
    lo, hi = C.c_int(), C.c_int()
    lib().ora_stretch_levels(a, H, W, W, hist, C.byref(lo), C.byref(hi))
    return lo.value, hi.value, hist


def stretch(img: np.ndarray) -> np.ndarray:
    """The stretched image clip((v - low)/(high - low), 0, 1) in FP64 (0
    where high = low)."""
    a = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = a.shape
    out = np.zeros((H, W), np.float64)
    lo, hi = C.c_int(), C.c_int()
    lib().ora_stretch(a, H, W, W, out, C.byref(lo), C.byref(hi))
    return out


def gauss_stack(img, sigmas, truncate: float = 4.0) -> np.ndarray:
    """Gaussian planes L_k = G_{sigma_k} * I (K x H x W, FP64)."""
    I = to_f64(img)
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    H, W = I.shape
    out = np.zeros((len(sg), H, W), np.float64)
    lib().ora_gauss_stack(I, H, W, len(sg), sg, float(truncate), out)
    return out


def dog_criterion(L: np.ndarray, sigmas, tau: float = -np.inf) -> dict:
    """The paper's criterion (equations "dog" and "argmax", Algorithm 1) on
    Gaussian planes L: M = max over i of t_i (L_{i+1} - L_i), idx its first
    argmax, and the pixels whose M exceeds tau and equals its 3x3 maximum.
    Returns dict(M, idx, yxk, count)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    K, H, W = L.shape
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    M = np.zeros((H, W), np.float64)
    idx = np.zeros((H, W), np.int32)
    cap = H * W
    yxk = np.zeros((cap, 3), np.int32)
    n = lib().ora_dog_criterion(L, H, W, K, sg, float(tau), M, idx, yxk, cap)
    return dict(M=M, idx=idx, yxk=yxk[:n], count=int(n))


def detect(img, sigmas, truncate: float = 4.0, tau: float = 0.1, theta: float = 0.5,
           polarity: int = 0, stack: np.ndarray | None = None) -> dict:
    """Whole detector: stack, candidates, prune, count and density.

    The focus criterion is the number of surviving blobs (|C|, section 3 and
    Algorithm 1); density is that count per megapixel."""
    sg = np.asarray(sigmas, dtype=np.float64)
    if stack is None:
        stack = log_stack(img, sg, truncate, polarity)
    K, H, W = stack.shape
    ykx, resp = candidates(stack, tau)
    keep = prune(ykx, sg, theta) if theta < 1.0 else np.ones(len(ykx), dtype=bool)
    blobs = ykx[keep]
    return dict(stack=stack, cand=ykx, cand_resp=resp, keep=keep, blobs=blobs,
                blob_resp=resp[keep], blob_sigma=sg[blobs[:, 2]] if len(blobs) else np.zeros(0),
                count=int(keep.sum()), density=float(keep.sum()) * 1e6 / (H * W))


# ----------------------------------------------------------------------------
# soft focus score
# ----------------------------------------------------------------------------

def _radii(sigmas, truncate, radii):
    if radii is None:
        radii = [radius(s, truncate) for s in sigmas]
    return np.ascontiguousarray(np.asarray(radii, dtype=np.int32))


def soft_score(imgs, sigmas, beta: float, tau: float, truncate: float = 4.0,
               radii=None) -> np.ndarray:
    """S_b = mean over scales and pixels of softplus(beta (|r| - tau))."""
    I = np.ascontiguousarray(np.asarray(imgs, dtype=np.float64))
    if I.ndim == 2:
        I = I[None]
    Bn, H, W = I.shape
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    out = np.zeros(Bn)
    lib().ora_soft_score(I, Bn, H, W, len(sg), sg, _radii(sg, truncate, radii),
                         float(beta), float(tau), out)
    return out


def soft_score_grad(imgs, sigmas, beta: float, tau: float, gbar=None, truncate: float = 4.0,
                    radii=None):
    """(dS/dI, dS/dsigma) contracted with upstream gradients gbar[b]."""
    I = np.ascontiguousarray(np.asarray(imgs, dtype=np.float64))
    if I.ndim == 2:
        I = I[None]
    Bn, H, W = I.shape
    sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    gb = np.ascontiguousarray(np.ones(Bn) if gbar is None else np.asarray(gbar, np.float64))
    dI = np.zeros((Bn, H, W))
    ds = np.zeros(len(sg))
    lib().ora_soft_score_grad(I, Bn, H, W, len(sg), sg, _radii(sg, truncate, radii),
                              float(beta), float(tau), gb, dI, ds)
    return dI, ds
