"""Moments as image hashes for dataset de-duplication (Sec. 2.7).

eq. (16): image k's hash at order l is taken from its order-l moments; here
the vector of magnitudes |Z_lm|, m = l mod 2 .. l step 2, which quarter turns
and mirror images of the content leave unchanged.  Two images agree at order
l when their hashes differ by at most ``rtol`` times the larger one's largest
entry (max norm; exact copies agree exactly, turned or mirrored copies up to
rounding).  eq. (17): images that agree at every listed order have the same
content; the groups are the classes of that relation.

The moments come from the library (all orders up to max(orders) in one
zm_moments launch per chunk of frames); candidate pairs come from sorting
every image by one hash entry and sweeping a window of the largest allowed
difference, then each candidate is checked at every order.
"""
from __future__ import annotations

import numpy as np


def _hashes(Z: np.ndarray, orders) -> list:
    """Z: [K][M_tot] complex (canonical order).  Returns one [K][len] array of
    magnitudes per order."""
    from . import index
    out = []
    for l in orders:
        cols = [index(l, m) for m in range(l % 2, l + 1, 2)]
        out.append(np.abs(Z[:, cols]))
    return out


def groups_from_moments(Z: np.ndarray, orders, rtol: float = 1e-5) -> list:
    """Groups (sorted lists of >= 2 image indices) of images whose order-l
    hashes agree for every l in ``orders``."""
    K = Z.shape[0]
    if K < 2:
        return []
    hs = _hashes(Z, orders)
    scale = [h.max(axis=1) for h in hs]  # largest entry of each image's hash
    # sweep on the entry with the largest spread of the first order
    h0 = hs[0]
    c = int(np.argmax(h0.std(axis=0))) if h0.shape[1] > 1 else 0
    key = h0[:, c]
    order = np.argsort(key, kind="stable")
    window = rtol * float(scale[0].max())  # no agreeing pair differs by more in any entry
    parent = np.arange(K)

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for p in range(K):
        i = order[p]
        q = p + 1
        while q < K and key[order[q]] - key[i] <= window:
            j = order[q]
            ok = True
            for h, s in zip(hs, scale):
                if np.max(np.abs(h[i] - h[j])) > rtol * max(s[i], s[j]):
                    ok = False
                    break
            if ok:
                ri, rj = root(i), root(j)
                if ri != rj:
                    parent[max(ri, rj)] = min(ri, rj)
            q += 1
    classes = {}
    for k in range(K):
        classes.setdefault(root(k), []).append(k)
    return sorted(sorted(v) for v in classes.values() if len(v) > 1)


def find_duplicates(frames, orders=(16, 20), rtol: float = 1e-5, dtype: str = "f32", chunk: int = 256,
                    plan=None, stream=None):
    """Groups of frames with the same content among ``frames`` ([K, H, W]
    float32 CUDA tensor, or a list of [H, W] tensors of one size).  Moments of
    every order up to max(orders) are computed on the GPU, ``chunk`` frames
    per launch.  Returns (groups, Z) with Z the [K][M_tot] complex moments."""
    import torch

    from . import Plan, as_complex
    if isinstance(frames, (list, tuple)):
        frames = torch.stack(list(frames))
    K, H, W = frames.shape
    nmax = max(orders)
    if plan is None:
        plan = Plan(nmax, H, W, dtype=dtype)
    ws = plan.workspace(min(chunk, K))
    Z = torch.empty(K, plan.num_moments, 2, dtype=plan._real_dtype(), device=frames.device)
    for s in range(0, K, chunk):
        e = min(K, s + chunk)
        plan.moments(frames[s:e].contiguous(), out=Z[s:e], workspace=ws, stream=stream)
    Zc = as_complex(Z).cpu().numpy().astype(np.complex128)
    return groups_from_moments(Zc, orders, rtol), Zc
