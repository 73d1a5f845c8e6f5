"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
binding, run the oracle on the same seeded input, compare.

Comparison rules (the stated tolerances are in the tests):
  * LoG stack: per-plane max |R_gpu - R_oracle| / max |R_oracle|.
  * Candidates and blobs: the oracle's ambiguity map marks the voxels whose
    candidate decision lies within eps of the threshold or of a window
    neighbour; every other decision must agree exactly.  At ambiguous voxels
    either decision is correct, so the GPU's decision is checked against the
    GPU's own stack values instead.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle

EPS_DECISION = 1e-4


def gpu_detect(plan, img_np: np.ndarray, return_stack: bool = True, capacity=None):
    dev = plan.device
    t = torch.from_numpy(np.ascontiguousarray(img_np)).to(dev)
    d = plan.detect(t, capacity=capacity, return_stack=return_stack)
    yxk, sig, resp = d.numpy()
    st = d.stack.cpu().numpy() if return_stack else None
    return dict(yxk=yxk.astype(np.int64), sigma=sig, resp=resp, count=d.count,
                n_cand=d.n_candidates, flags=d.flags, stack=st)


def plane_rel_err(st_gpu: np.ndarray, st_ora: np.ndarray) -> np.ndarray:
    err = np.abs(st_gpu.astype(np.float64) - st_ora).reshape(len(st_ora), -1).max(1)
    ref = np.abs(st_ora).reshape(len(st_ora), -1).max(1)
    return err / np.maximum(ref, 1e-300)


def window_max_excl(st: np.ndarray) -> np.ndarray:
    """Largest other voxel of every 3x3x3 window (-inf padding), for the
    self-consistency check of ambiguous decisions."""
    from scipy.ndimage import maximum_filter
    fp = np.ones((3, 3, 3), bool)
    fp[1, 1, 1] = False
    return maximum_filter(st, footprint=fp, mode="constant", cval=-np.inf)


def compare_candidates(gpu_stack: np.ndarray, gpu_cand: set, ora_stack: np.ndarray,
                       ora_cand: set, tau32: float, eps: float = EPS_DECISION,
                       rows=None, row0: int = 0):
    """Returns (n_ambiguous, n_disagreeing).  Asserts exact agreement on
    unambiguous voxels and, at ambiguous ones, that the GPU's decision follows
    from its own stack.  Stacks may be row bands starting at image row `row0`;
    candidate sets hold image coordinates (y, x, k); only rows in `rows`
    (an image-row range, default all) are compared."""
    K, H, W = ora_stack.shape
    lo, hi = (row0, row0 + H) if rows is None else rows
    _, amb = oracle.ambiguous(ora_stack, tau32, eps, mask=True)
    ka, ya, xa = np.nonzero(amb)
    ya = ya + row0
    sel = (ya >= lo) & (ya < hi)
    ka, ya, xa = ka[sel], ya[sel], xa[sel]
    amb_set = set(zip(ya.tolist(), xa.tolist(), ka.tolist()))
    inrows = lambda c: {t for t in c if lo <= t[0] < hi}  # noqa: E731
    g, o = inrows(gpu_cand), inrows(ora_cand)
    diff = g ^ o
    bad = [d for d in diff if d not in amb_set]
    assert not bad, f"decisions differ at unambiguous voxels (y, x, k): {sorted(bad)[:10]}"
    if len(ka):
        wm = window_max_excl(gpu_stack)
        v = gpu_stack[ka, ya - row0, xa]
        is_c = (v > np.float32(tau32)) & (v >= wm[ka, ya - row0, xa])
        got = np.array([(y, x, k) in g for y, x, k in zip(ya.tolist(), xa.tolist(), ka.tolist())])
        assert np.array_equal(is_c, got), "GPU decision inconsistent with its own stack"
    return len(amb_set), len(diff)


def as_set(yxk) -> set:
    return set(map(tuple, np.asarray(yxk).reshape(-1, 3).tolist()))


def kink_bound(img: np.ndarray, sig, beta: float, tau: float, gbar: float, eps: float = 1e-5):
    """Per-pixel bound on how much the image gradient of the soft score may
    legitimately differ between two evaluations whose responses agree to
    within eps.  Only voxels with |r| <= eps can take the other sign of r;
    there the cotangent c = w sigma^2 changes by at most
    2 beta sigmoid(beta (eps - tau)) |gbar| sigma^2 / (K H W), and the change
    reaches dI through the Laplacian operator, bounded by the same operator
    with absolute taps."""
    from scipy.ndimage import correlate1d
    I = np.asarray(img, dtype=np.float64)
    H, W = I.shape
    K = len(sig)
    r = oracle.log_stack(I, sig, polarity=1)
    dw = 2.0 * beta / (1.0 + np.exp(-beta * (eps - tau))) * abs(gbar) / (K * H * W)
    out = np.zeros((H, W))
    for k, s in enumerate(sig):
        m = (np.abs(r[k]) <= eps).astype(np.float64) * dw * s * s
        if not m.any():
            continue
        g, h = oracle.taps(s, oracle.radius(s))
        ag, ah = np.abs(g), np.abs(h)
        out += correlate1d(correlate1d(m, ag, axis=1, mode="reflect"), ah, axis=0, mode="reflect")
        out += correlate1d(correlate1d(m, ah, axis=1, mode="reflect"), ag, axis=0, mode="reflect")
    return out


def strip_prune(cand: np.ndarray, sigmas, theta: float, H: int, step: int = 128,
                margin: int = 32) -> np.ndarray:
    """The oracle's one-shot prune of a canonical (y, x, k) candidate list,
    run strip by strip: a candidate's fate depends only on candidates closer
    than r_a + r_b, so each `step`-row strip is pruned together with the
    candidates `margin` rows around it (margin must exceed that reach) and
    keeps the decisions of its own rows.  Returns the kept records in order."""
    out = []
    for s0 in range(0, H, step):
        sel = (cand[:, 0] >= s0 - margin) & (cand[:, 0] < s0 + step + margin)
        sub = cand[sel]
        keep = oracle.prune(sub[:, :3], sigmas, theta)
        own = (sub[:, 0] >= s0) & (sub[:, 0] < s0 + step)
        out.append(sub[keep & own])
    return np.concatenate(out) if out else cand[:0]


def own_maxima(stack: np.ndarray, tau: float) -> np.ndarray:
    """Canonical (y, x, k) list of the voxels of `stack` (K x H x W, the
    GPU's own values) that equal the maximum of their 3x3x3 window (-inf
    outside the volume) and exceed tau: the candidate rule applied to the
    same FP32 values, so the GPU's candidate list must equal it exactly."""
    from scipy.ndimage import maximum_filter
    mx = maximum_filter(stack, size=3, mode="constant", cval=-np.inf)
    mask = (stack == mx) & (stack > np.float32(tau))
    del mx
    y, x, k = np.nonzero(mask.transpose(1, 2, 0))
    return np.stack([y, x, k], axis=1).astype(np.int64)
