"""High-order stability of the radial tables (Sec. 3.1, Fig. 1): orthogonality
of R_nm on Gauss-Legendre rings, per order, for the FP64 table of eq. (7) and
for the number formats the projection holds it in.

The Zernike radial polynomials are orthogonal on [0, 1] with weight rho,
int R_nm R_n'm rho drho = delta_nn' / (2(n+1)) (Sec. 2), and Gauss-Legendre
rings with R > n_max integrate the products exactly, so

    E(n) = max_n' | 2(n+1) sum_r w_r R_nm(rho_r) R_n'm(rho_r) - delta_nn' |

(over m and the n' of the same m) measures how far a table of R_nm values is
from the exact polynomials.  The paper plots an orthogonality measure of
this kind to show that the FFT route stays stable to order 500 where the
q-recursive route fails above 150 (Sec. 3.1, Fig. 1; the figure's values
are not in the text).

Besides the FP64 table itself, E(n) is evaluated for the table as the
projection operand stores it: the folded value t = c_n w_r R_nm(rho_r),
c_n = 2(n+1) / (A eps_m), rounded to FP32, split into hi + lo bfloat16
(hi = RNE(t), lo = RNE(t - hi), each through FP32), or scaled per row by a
power of two into [2^14, 2^15) and split into hi + lo IEEE half (each
rounded once from FP64, to nearest even); the value
seen by the projection is hi + lo (scaled back), divided by c_n w_r again to
give R.  The library builds the operand only for plans it computes moments
for (n_max <= 255); ``operand_effective`` reads it from the device there,
and ``split_effective`` forms the same values on the host from the FP64
table for higher orders (a GPU test checks that the two agree bit for bit).
"""
from __future__ import annotations

import ctypes

import numpy as np


def _bf16_rne(x32: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (rounded.astype(np.uint32) << 16).view(np.float32)


def fold_factors(plan) -> np.ndarray:
    """c_n w_r for every stored (n, m) and ring: [num_moments][R] FP64."""
    pairs = [(n, m) for n in range(plan.n_max + 1) for m in range(n % 2, n + 1, 2)]
    _, w = plan.ring_nodes()
    c = np.array([2.0 * (n + 1) / (plan.angles * (2.0 if (plan.neumann and m == 0) else 1.0)) for n, m in pairs])
    return c[:, None] * w[None, :]


def split_effective(table: np.ndarray, fold: np.ndarray, fmt: str) -> np.ndarray:
    """R values as the projection operand holds them, formed on the host from
    the FP64 table by the operand's rounding rule ("f64", "f32", "bf16x2",
    "f16x2")."""
    t = fold * table
    if fmt == "f64":
        eff = t
    elif fmt == "f32":
        eff = t.astype(np.float32).astype(np.float64)
    elif fmt == "bf16x2":
        hi = _bf16_rne(t.astype(np.float32)).astype(np.float64)
        lo = _bf16_rne((t - hi).astype(np.float32)).astype(np.float64)
        eff = hi + lo
    elif fmt == "f16x2":
        mx = np.max(np.abs(t), axis=1)
        ex = np.frexp(mx)[1]
        e = np.where(mx > 0, 15 - ex, 0)
        sc = np.ldexp(1.0, e)[:, None]
        ts = t * sc
        hi = ts.astype(np.float16).astype(np.float64)
        lo = (ts - hi).astype(np.float16).astype(np.float64)
        eff = (hi + lo) * np.ldexp(1.0, -e)[:, None]
    else:
        raise ValueError(fmt)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(fold != 0, eff / fold, 0.0)


def operand_effective(plan) -> np.ndarray:
    """The device operand of a plan (n_max <= 255) decoded to R values,
    [num_moments][R] FP64 (zm_operand_table)."""
    from . import _check, _lib
    out = np.empty((plan.num_moments, plan.rings), dtype=np.float64)
    _check(_lib.zm_operand_table(plan.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
           "zm_operand_table")
    return out / fold_factors(plan)


def orthogonality(R: np.ndarray, n_max: int, w: np.ndarray) -> np.ndarray:
    """E(n) for n = 0..n_max of a table R [num_moments][rings] on rings with
    weights w (exact for the products when the rings are Gauss-Legendre
    with R > n_max)."""
    pairs = [(n, m) for n in range(n_max + 1) for m in range(n % 2, n + 1, 2)]
    ns = np.array([p[0] for p in pairs])
    ms = np.array([p[1] for p in pairs])
    worst = np.zeros(n_max + 1)
    for m in range(n_max + 1):
        idx = np.nonzero(ms == m)[0]
        G = (R[idx] * w[None, :]) @ R[idx].T * 2.0 * (ns[idx][:, None] + 1)
        err = np.max(np.abs(G - np.eye(len(idx))), axis=1)
        worst[ns[idx]] = np.maximum(worst[ns[idx]], err)
    return worst


def sweep(plan, formats=("f64", "f32", "bf16x2", "f16x2"), band: int = 50) -> dict:
    """E(n) of the plan's FP64 table (read from the device) and of its
    operand formats, reduced to the maximum per band of `band` orders."""
    table = plan.radial_table()
    _, w = plan.ring_nodes()
    fold = fold_factors(plan)
    out = {"n_max": plan.n_max, "rings": plan.rings, "band": band, "bands": [], "max": {}}
    curves = {fmt: orthogonality(split_effective(table, fold, fmt) if fmt != "f64" else table, plan.n_max, w)
              for fmt in formats}
    for b in range(0, plan.n_max + 1, band):
        row = {"n": [b, min(plan.n_max, b + band - 1)]}
        for fmt, E in curves.items():
            row[fmt] = float(E[b:b + band].max())
        out["bands"].append(row)
    for fmt, E in curves.items():
        out["max"][fmt] = float(E.max())
    out["curves"] = {fmt: E for fmt, E in curves.items()}
    return out
