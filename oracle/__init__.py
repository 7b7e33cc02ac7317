"""FP64 CPU oracle for Zernike moments -- TEST INFRASTRUCTURE, not the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2304_14492_amd``) and neither imports the other; both receive their
inputs from the seeded generators in ``synth``.

What it computes, each function citing the paper (Al-Rawi, arXiv 2304.14492):
  * ``zrp`` / ``zrp_table``      -- eq. (2), evaluated exactly (big integers),
  * ``ring_grid``                -- the radial quadrature nodes/weights of eq. (1),
  * ``resample``                 -- the polar image f^ of eq. (1) (Sec. 2.5, bilinear),
  * ``angular_dft``              -- the angular sum of eq. (1), a plain DFT,
  * ``radial_sum``               -- the radial sum of eq. (1) / eq. (14),
  * ``moments``                  -- eq. (1) end to end on the polar grid,
  * ``cartesian``                -- eq. (3) with eq. (5) (sanity check only),
  * ``reconstruct_*``            -- eq. (9),
  * ``recon_error``              -- eq. (13).

Readings of the paper that these functions take are listed in the module
docstrings below; the pins that tie this oracle to the paper and to the
mathematics live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zm_oracle.c")
# ZM_ORACLE_SO names another build of the same C source (the sanitizer run of
# the CPU tests loads one built with -fsanitize=address,undefined)
_SO = os.environ.get("ZM_ORACLE_SO") or os.path.join(_HERE, "_zm_oracle.so")
_lib_handle = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint64)
        L.zmo_zrp_pairs.argtypes = [ctypes.c_int, ip, ip, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_int, up, up, ip, dp]
        L.zmo_zrp_pairs.restype = ctypes.c_int
        L.zmo_num_moments.argtypes = [ctypes.c_int]
        L.zmo_num_moments.restype = ctypes.c_int
        L.zmo_resample.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.zmo_resample.restype = None
        L.zmo_angular_dft.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp]
        L.zmo_angular_dft.restype = None
        L.zmo_radial_sum.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ip,
                                     dp, dp, ctypes.c_int, dp]
        L.zmo_radial_sum.restype = None
        L.zmo_cartesian.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.zmo_cartesian.restype = ctypes.c_int
        L.zmo_cartesian_one.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.zmo_cartesian_one.restype = ctypes.c_int
        L.zmo_reconstruct.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.zmo_reconstruct.restype = None
        _lib_handle = L
    return _lib_handle


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# Moment enumeration (Sec. 2: n >= 0, |m| <= n, n - |m| even; Z_{n,-m} = Z_nm*
# so only m >= 0 is stored).  Canonical order: n ascending, then m ascending.
# ---------------------------------------------------------------------------
def pairs(nmax: int):
    return [(n, m) for n in range(nmax + 1) for m in range(n % 2, n + 1, 2)]


def num_moments(nmax: int) -> int:
    return len(pairs(nmax))


# ---------------------------------------------------------------------------
# Radial quadrature of eq. (1): int_0^1 g(rho) rho drho ~= sum_r w_r g(rho_r).
# "midpoint": rho_r = (2r+1)/(2R), w_r = rho_r / R  (uniform rings, Sec. 2.5).
# "gauss_legendre": Gauss-Legendre nodes on [0, 1], w_r = (w_GL / 2) rho_r.
# Each grid also carries an exact rational form of rho_r^2 = a_r / b with
# b common to all rings (a = ax*ay*2^ash, b = bx*by*2^bsh), for eq. (2).
# ---------------------------------------------------------------------------
def ring_grid(R: int, rule: str = "midpoint") -> dict:
    if rule == "midpoint":
        p = np.arange(R, dtype=np.int64) * 2 + 1
        rho = np.array([float(Fraction(int(pi), 2 * R)) for pi in p])
        w = np.array([float(Fraction(int(pi), 2 * R * R)) for pi in p])
        ax = p.astype(np.uint64)
        return dict(rho=rho, w=w, ax=ax, ay=ax.copy(), ash=np.zeros(R, np.int32),
                    bx=2 * R, by=2 * R, bsh=0, rule=rule)
    if rule == "gauss_legendre":
        x, wg = np.polynomial.legendre.leggauss(R)
        rho = 0.5 * (x + 1.0)
        return node_grid(rho, 0.5 * wg * rho, rule)
    raise ValueError(rule)


def node_grid(rho, w, rule: str = "nodes") -> dict:
    """A ring grid at given FP64 nodes in (0, 1] (and weights), with the exact
    rational form of each node: rho_r = M_r 2^(e_r - 53), rho_r^2 over the
    common denominator 2^(2L)."""
    rho = np.asarray(rho, dtype=np.float64)
    mants, shifts = [], []
    for v in rho:
        fm, e = math.frexp(float(v))
        mants.append(int(fm * (1 << 53)))
        shifts.append(53 - e)
    L = max(shifts)
    ax = np.array(mants, dtype=np.uint64)
    ash = np.array([2 * (L - s) for s in shifts], dtype=np.int32)
    return dict(rho=rho, w=np.asarray(w, dtype=np.float64), ax=ax, ay=ax.copy(), ash=ash, bx=1, by=1, bsh=2 * L,
                rule=rule)


def zrp(plist, grid: dict) -> np.ndarray:
    """Eq. (2) evaluated exactly at every ring of ``grid`` for each (n, m) in
    ``plist``; returns [len(plist)][R] FP64 (each value rounded once)."""
    L = _lib()
    ns = np.ascontiguousarray([n for n, _ in plist], dtype=np.int32)
    ms = np.ascontiguousarray([m for _, m in plist], dtype=np.int32)
    R = len(grid["rho"])
    out = np.empty((len(plist), R), dtype=np.float64)
    ax = np.ascontiguousarray(grid["ax"], dtype=np.uint64)
    ay = np.ascontiguousarray(grid["ay"], dtype=np.uint64)
    ash = np.ascontiguousarray(grid["ash"], dtype=np.int32)
    rc = L.zmo_zrp_pairs(len(plist), _p(ns, ctypes.c_int), _p(ms, ctypes.c_int),
                         int(grid["bx"]), int(grid["by"]), int(grid["bsh"]), R,
                         _p(ax, ctypes.c_uint64), _p(ay, ctypes.c_uint64), _p(ash, ctypes.c_int),
                         _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("invalid (n, m) pair")
    return out


def zrp_rational(plist, a_list, b: int) -> np.ndarray:
    """Eq. (2) exactly at points rho^2 = a/b (a, b non-negative integers < 2^64)."""
    L = _lib()
    ns = np.ascontiguousarray([n for n, _ in plist], dtype=np.int32)
    ms = np.ascontiguousarray([m for _, m in plist], dtype=np.int32)
    ax = np.ascontiguousarray(a_list, dtype=np.uint64)
    ay = np.ones_like(ax)
    ash = np.zeros(len(ax), dtype=np.int32)
    out = np.empty((len(plist), len(ax)), dtype=np.float64)
    rc = L.zmo_zrp_pairs(len(plist), _p(ns, ctypes.c_int), _p(ms, ctypes.c_int), int(b), 1, 0, len(ax),
                         _p(ax, ctypes.c_uint64), _p(ay, ctypes.c_uint64), _p(ash, ctypes.c_int),
                         _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("invalid (n, m) pair")
    return out


def zrp_table(nmax: int, grid: dict) -> np.ndarray:
    return zrp(pairs(nmax), grid)


# ---------------------------------------------------------------------------
# Eq. (1) on the polar grid.
# ---------------------------------------------------------------------------
def resample(frame: np.ndarray, R: int, A: int, rho: np.ndarray) -> np.ndarray:
    """Bilinear pixel -> polar resampling (Sec. 2.5); returns f^ [R][A] FP64.
    Unit disk = inscribed disk of radius D/2 px centred at ((W-1)/2, (H-1)/2);
    x right, y up, theta_a = 2 pi a / A counter-clockwise; taps outside the
    frame are 0."""
    f = np.ascontiguousarray(frame, dtype=np.float64)
    H, W = f.shape
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    out = np.empty((R, A), dtype=np.float64)
    _lib().zmo_resample(_p(f, ctypes.c_double), H, W, R, A, _p(rho, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def angular_dft(fhat: np.ndarray, mlist) -> np.ndarray:
    """G[r][j] = sum_a f^[r][a] exp(-i m_j 2 pi a / A): the angular integral of eq. (1)."""
    fh = np.ascontiguousarray(fhat, dtype=np.float64)
    R, A = fh.shape
    ml = np.ascontiguousarray(mlist, dtype=np.int32)
    G = np.empty((R, len(ml), 2), dtype=np.float64)
    _lib().zmo_angular_dft(_p(fh, ctypes.c_double), R, A, len(ml), _p(ml, ctypes.c_int), _p(G, ctypes.c_double))
    return G[..., 0] + 1j * G[..., 1]


def radial_sum(G: np.ndarray, mlist, plist, A: int, table: np.ndarray, w: np.ndarray, neumann: bool) -> np.ndarray:
    """Z_nm = (n+1)/(pi eps_m) (2 pi / A) sum_r w_r R_nm(rho_r) G[r][m]  -- eq. (1) / eq. (14)."""
    R = G.shape[0]
    col = {int(m): j for j, m in enumerate(mlist)}
    ns = np.ascontiguousarray([n for n, _ in plist], dtype=np.int32)
    ms = np.ascontiguousarray([m for _, m in plist], dtype=np.int32)
    cols = np.ascontiguousarray([col[m] for _, m in plist], dtype=np.int32)
    Gr = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1), dtype=np.float64)
    tb = np.ascontiguousarray(table, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    Z = np.empty((len(plist), 2), dtype=np.float64)
    _lib().zmo_radial_sum(_p(Gr, ctypes.c_double), R, len(mlist), A, len(plist), _p(ns, ctypes.c_int),
                          _p(ms, ctypes.c_int), _p(cols, ctypes.c_int), _p(tb, ctypes.c_double),
                          _p(ww, ctypes.c_double), int(bool(neumann)), _p(Z, ctypes.c_double))
    return Z[:, 0] + 1j * Z[:, 1]


def moments_polar(fhat: np.ndarray, plist, grid: dict, neumann: bool = False, table=None) -> np.ndarray:
    """Eq. (1) / (14) from a polar image f^ [R][A] (bypasses the resampler)."""
    A = fhat.shape[1]
    mlist = sorted({m for _, m in plist})
    if table is None:
        table = zrp(plist, grid)
    G = angular_dft(fhat, mlist)
    return radial_sum(G, mlist, plist, A, table, grid["w"], neumann)


def moments(frame: np.ndarray, nmax: int, R: int, A: int, neumann: bool = False, rule: str = "midpoint",
            plist=None, table=None) -> np.ndarray:
    """All (or the listed) Zernike moments of eq. (1) (eq. (14) with ``neumann``)
    of one frame on the R x A polar grid, complex FP64 in canonical order."""
    grid = ring_grid(R, rule)
    if plist is None:
        plist = pairs(nmax)
    fhat = resample(frame, R, A, grid["rho"])
    return moments_polar(fhat, plist, grid, neumann, table)


# ---------------------------------------------------------------------------
# Eq. (3) + (5) / eq. (6), (14): Cartesian pixel sum.
# ---------------------------------------------------------------------------
def cartesian_moment(frame: np.ndarray, n: int, m: int, neumann: bool = False) -> complex:
    """One moment Z_nm of the Cartesian pixel sum (eq. (6); eq. (14) with
    ``neumann``), R_nm exact (eq. (2), big-integer) at every disk pixel centre;
    m < 0 through Z_{n,-m} = conj(Z_nm)."""
    f = np.ascontiguousarray(frame, dtype=np.float64)
    H, W = f.shape
    Z = np.empty(2, dtype=np.float64)
    rc = _lib().zmo_cartesian_one(_p(f, ctypes.c_double), H, W, int(n), int(m), int(bool(neumann)),
                                  _p(Z, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"bad moment (n, m) = ({n}, {m})")
    return complex(Z[0], Z[1])


def cartesian(frame: np.ndarray, nmax: int, neumann: bool = False) -> np.ndarray:
    f = np.ascontiguousarray(frame, dtype=np.float64)
    H, W = f.shape
    mt = num_moments(nmax)
    Z = np.empty((mt, 2), dtype=np.float64)
    rc = _lib().zmo_cartesian(_p(f, ctypes.c_double), H, W, nmax, int(bool(neumann)), _p(Z, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("zmo_cartesian failed")
    return Z[:, 0] + 1j * Z[:, 1]


# ---------------------------------------------------------------------------
# Eq. (9) reconstruction and eq. (13) error.
# ---------------------------------------------------------------------------
def reconstruct(Z: np.ndarray, nmax: int, Rvals: np.ndarray, theta: np.ndarray, neumann: bool = False,
                one_sided: bool = False) -> np.ndarray:
    """f~ at points with R_nm values Rvals [M_tot][count] and angles theta [count]."""
    Zr = np.ascontiguousarray(np.stack([Z.real, Z.imag], axis=-1), dtype=np.float64)
    Rv = np.ascontiguousarray(Rvals, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(th.shape[0], dtype=np.float64)
    _lib().zmo_reconstruct(_p(Zr, ctypes.c_double), nmax, int(bool(neumann)), int(bool(one_sided)), th.shape[0],
                           _p(Rv, ctypes.c_double), _p(th, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def disk_pixels(H: int, W: int):
    """Pixel centres with rho <= 1: (mask [H][W], integer rho^2 numerators P, D^2, theta)."""
    D = min(H, W)
    X = 2 * np.arange(W, dtype=np.int64) - (W - 1)
    Y = (H - 1) - 2 * np.arange(H, dtype=np.int64)
    P = X[None, :] ** 2 + Y[:, None] ** 2
    mask = P <= D * D
    th = np.arctan2(np.broadcast_to(Y[:, None], (H, W)), np.broadcast_to(X[None, :], (H, W)))
    return mask, P[mask], D * D, th[mask]


def reconstruct_cartesian(Z: np.ndarray, H: int, W: int, nmax: int, neumann: bool = False,
                          one_sided: bool = False) -> np.ndarray:
    """Eq. (9) at the pixel centres inside the disk (0 outside)."""
    mask, P, b, th = disk_pixels(H, W)
    Rv = zrp_rational(pairs(nmax), P, b)
    vals = reconstruct(Z, nmax, Rv, th, neumann, one_sided)
    out = np.zeros((H, W), dtype=np.float64)
    out[mask] = vals
    return out


def reconstruct_polar(Z: np.ndarray, nmax: int, R: int, A: int, neumann: bool = False,
                      rule: str = "midpoint", one_sided: bool = False) -> np.ndarray:
    """Eq. (9) at the polar nodes (rho_r, theta_a); returns [R][A]."""
    grid = ring_grid(R, rule)
    tab = zrp_table(nmax, grid)  # [M][R]
    th = 2.0 * np.pi * np.arange(A) / A
    Rv = np.repeat(tab, A, axis=1)  # point (r, a) -> column r*A + a
    thv = np.tile(th, R)
    return reconstruct(Z, nmax, Rv, thv, neumann, one_sided).reshape(R, A)


def recon_error(f: np.ndarray, ft: np.ndarray, mask: np.ndarray) -> dict:
    """Eq. (13): sum_disk (f - f~)^2 / (f_max^2 * count_disk); also sqrt (NRMSE)
    and -10 log10 (a PSNR in dB); eq. (10) for context; eq. (12):
    sum_disk (f - f~)^2 / f^2 over the pixels with f != 0 (the measure is
    singular where f = 0; ``zeros`` counts the disk pixels it leaves out)."""
    fd = f[mask].astype(np.float64)
    td = ft[mask].astype(np.float64)
    fmax = float(np.max(np.abs(fd))) if fd.size else 0.0
    sse = float(np.sum((fd - td) ** 2))
    eps = sse / (fmax * fmax * fd.size) if fmax > 0 else float("nan")
    e1 = sse / float(np.sum(fd * fd)) if np.any(fd) else float("nan")
    nz = fd != 0.0
    e2 = float(np.sum((fd[nz] - td[nz]) ** 2 / (fd[nz] * fd[nz])))
    return dict(eps13=eps, nrmse=math.sqrt(eps) if eps == eps else eps,
                psnr_db=-10.0 * math.log10(eps) if eps and eps > 0 else float("inf"), eps10=e1,
                eps12=e2, zeros=int(np.count_nonzero(~nz)))


def minmax(ft: np.ndarray, f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Min-max renormalisation of a reconstruction (Sec. 2.3, Sec. 3): the
    affine map taking [min f~, max f~] over the disk onto [min f, max f] of
    the original band; pixels outside the disk are left at 0."""
    lo_t, hi_t = float(ft[mask].min()), float(ft[mask].max())
    lo, hi = float(f[mask].min()), float(f[mask].max())
    out = np.zeros_like(ft, dtype=np.float64)
    scale = (hi - lo) / (hi_t - lo_t) if hi_t > lo_t else 0.0
    out[mask] = (ft[mask] - lo_t) * scale + lo
    return out


# ---------------------------------------------------------------------------
# Sec. 2.7, eq. (16)-(17): moments as image hashes for de-duplication.
# ---------------------------------------------------------------------------
def dedup_groups(Z: np.ndarray, nmax: int, orders, rtol: float):
    """Groups of images with the same content, from their moment vectors Z
    ([K][M_tot] complex, canonical order, moments up to nmax).  For each order
    l in ``orders`` (eq. (16)) an image's hash is the vector of magnitudes
    |Z_lm|, m = l mod 2 .. l step 2 (unchanged by quarter turns and mirrors
    of the content); two images agree at order l when the hashes differ by at
    most rtol times the larger one's largest entry (max norm).  eq. (17): two
    images have the same content when they agree at every listed order; the
    groups are the classes of that relation closed transitively.  All pairs
    are compared (small sets).  Returns sorted lists of >= 2 indices."""
    K = len(Z)
    idx = {(n, m): i for i, (n, m) in enumerate(pairs(nmax))}
    hashes = []
    for k in range(K):
        hk = []
        for l in orders:
            hk.append([abs(Z[k][idx[(l, m)]]) for m in range(l % 2, l + 1, 2)])
        hashes.append(hk)
    parent = list(range(K))

    def root(a):
        while parent[a] != a:
            a = parent[a]
        return a

    for i in range(K):
        for j in range(i + 1, K):
            same = True
            for o in range(len(orders)):
                a, b = hashes[i][o], hashes[j][o]
                scale = max(max(a), max(b))
                if max(abs(x - y) for x, y in zip(a, b)) > rtol * scale:
                    same = False
                    break
            if same:
                parent[root(j)] = root(i)
    classes = {}
    for k in range(K):
        classes.setdefault(root(k), []).append(k)
    return sorted(sorted(c) for c in classes.values() if len(c) > 1)
