"""ctypes wrapper around the FP64 CPU oracle (``oracle/libagn_oracle.so``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct statement
of the light-curve iteration of Sartori et al. (2019), arXiv:1909.06374
(Sec. 2.1, Sec. 3.2.2, Eqs. 3, 4, A1, A2).  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU library
never does, and the two share no code.

All arrays are numpy float64 / uint32 on the host.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libagn_oracle.so")
_lib = None


class PsdParams(C.Structure):
    """Eq. 3 parameters; norm <= 0 selects the unit-variance normalisation."""
    _fields_ = [("norm", C.c_double), ("f_br", C.c_double),
                ("a_low", C.c_double), ("a_high", C.c_double)]


class ErdfParams(C.Structure):
    """Sharp broken power law in dN/dlog10(lambda) (Eq. 1 slope convention)."""
    _fields_ = [("u_min", C.c_double), ("u_max", C.c_double), ("u_br", C.c_double),
                ("d1", C.c_double), ("d2", C.c_double)]


def erdf_params(u_min=-4.0, u_max=0.0, u_br=-1.5, d1=0.4, d2=2.5):
    return ErdfParams(float(u_min), float(u_max), float(u_br), float(d1), float(d2))


class PdfParams(C.Structure):
    """General PDF of Sec. 2.1 step (ii): kind 0 sharp broken power law, 1 Eq. 1,
    2 Eq. 2 (log-normal); measure 0 dN/dlog10(lambda), 1 dN/dlambda."""
    _fields_ = [("kind", C.c_int32), ("measure", C.c_int32), ("u_min", C.c_double),
                ("u_max", C.c_double), ("u_star", C.c_double), ("d1", C.c_double),
                ("d2", C.c_double), ("sigma", C.c_double)]


def pdf_params(kind, measure=0, u_min=-3.75, u_max=0.5, u_star=math.log10(0.11), d1=0.47, d2=2.53,
               sigma=0.64):
    """Defaults: the Eq. 1 parameters of the reference simulation (Table 2)."""
    return PdfParams(int(kind), int(measure), float(u_min), float(u_max), float(u_star), float(d1),
                     float(d2), float(sigma))


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    d, i64, i32, u32, u64 = C.c_double, C.c_int64, C.c_int32, C.c_uint32, C.c_uint64
    pd, pu32, pi32 = C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.POINTER(C.c_int32)
    lib.agn_oracle_philox4x64.argtypes = [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
    lib.agn_oracle_philox4x64.restype = None
    lib.agn_oracle_uniform.argtypes = [u64, u32, u32, u64]
    lib.agn_oracle_uniform.restype = d
    lib.agn_oracle_psd_eq3.argtypes = [d, d, d, d, d]
    lib.agn_oracle_psd_eq3.restype = d
    lib.agn_oracle_psd_norm.argtypes = [C.POINTER(PsdParams), i64, d]
    lib.agn_oracle_psd_norm.restype = d
    lib.agn_oracle_psd_spectrum.argtypes = [C.POINTER(PsdParams), i64, d, u64, u32, pd]
    lib.agn_oracle_dft.argtypes = [pd, i64, C.c_int]
    lib.agn_oracle_rfft.argtypes = [pd, i64, pd]
    lib.agn_oracle_irfft.argtypes = [pd, i64, pd]
    lib.agn_oracle_replace.argtypes = [pd, pd, i64, pd]
    lib.agn_oracle_argsort.argtypes = [pd, i64, pu32]
    lib.agn_oracle_iterate.argtypes = [pd, pd, i64, i32, d, pd, pd, pi32, pu32]
    lib.agn_oracle_generate.argtypes = [C.POINTER(PsdParams), pd, i64, d, i32, d, u64, u32,
                                        pd, pd, pi32, pu32]
    lib.agn_oracle_periodogram.argtypes = [pd, i64, pd]
    lib.agn_oracle_erdf_bpl.argtypes = [C.POINTER(ErdfParams), i64, u64, u32, pd]
    lib.agn_oracle_erdf_bpl.restype = C.c_int
    lib.agn_oracle_pdf_draw.argtypes = [C.POINTER(PdfParams), i64, u64, u32, pd]
    lib.agn_oracle_pdf_draw.restype = C.c_int
    lib.agn_oracle_pdf_draw_at.argtypes = [C.POINTER(PdfParams), u64, u32, C.POINTER(C.c_int64), i64, pd]
    lib.agn_oracle_pdf_draw_at.restype = C.c_int
    pu64 = C.POINTER(C.c_uint64)
    lib.agn_oracle_lag_stats.argtypes = [pd, i64, C.POINTER(C.c_int64), i32, i32, pd, i32, d, pd, pu64, pu64]
    lib.agn_oracle_lag_stats.restype = C.c_int
    lib.agn_oracle_psd_fit.argtypes = [pd, pd, i64, d, d, d, pd]
    lib.agn_oracle_psd_fit.restype = C.c_int
    lib.agn_oracle_uniform_chain.argtypes = [u64, u32, u32, u64, u64]
    lib.agn_oracle_uniform_chain.restype = d
    lib.agn_oracle_pdf_slice.argtypes = [C.POINTER(PdfParams), i64, i32, i32, u64, u32, pd]
    lib.agn_oracle_pdf_slice.restype = C.c_int
    for name in ("psd_spectrum", "dft", "rfft", "irfft", "replace", "argsort",
                 "iterate", "generate", "periodogram"):
        getattr(lib, "agn_oracle_" + name).restype = C.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _chk(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pu32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def psd_params(norm=0.0, f_br=1.0, a_low=1.0, a_high=2.0):
    return PsdParams(float(norm), float(f_br), float(a_low), float(a_high))


def philox4x64(ctr, key):
    lib = _load()
    c = (C.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (C.c_uint64 * 4)()
    lib.agn_oracle_philox4x64(c, k, o)
    return [int(v) for v in o]


def uniform(seed, stream, curve_id, k):
    return _load().agn_oracle_uniform(int(seed), int(stream), int(curve_id), int(k))


def psd_eq3(f, A, f_br, a_low, a_high):
    return _load().agn_oracle_psd_eq3(float(f), float(A), float(f_br), float(a_low), float(a_high))


def psd_norm(params: PsdParams, n, dt):
    return _load().agn_oracle_psd_norm(C.byref(params), int(n), float(dt))


def psd_spectrum(params: PsdParams, n, dt, seed, curve_id=0):
    amp = np.full(n // 2 + 1, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_psd_spectrum(C.byref(params), int(n), float(dt), int(seed),
                                         int(curve_id), _pd(amp)), "psd_spectrum")
    return amp


def dft(z, sign=-1):
    """Unnormalised complex DFT (sign -1 forward, +1 inverse) of a complex array."""
    z = np.ascontiguousarray(z, dtype=np.complex128).copy()
    buf = z.view(np.float64)
    _chk(_load().agn_oracle_dft(_pd(buf), len(z), int(sign)), "dft")
    return z


def rfft(x):
    x = _f64(x)
    X = np.full(len(x) // 2 + 1, np.nan, dtype=np.complex128)
    _chk(_load().agn_oracle_rfft(_pd(x), len(x), _pd(X.view(np.float64))), "rfft")
    return X


def irfft(Y, n):
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    assert len(Y) == n // 2 + 1
    y = np.full(n, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_irfft(_pd(Y.view(np.float64)), int(n), _pd(y)), "irfft")
    return y


def replace(X, amp, n):
    X = np.ascontiguousarray(X, dtype=np.complex128)
    amp = _f64(amp)
    Y = np.full(X.shape, np.nan, dtype=np.complex128)
    _chk(_load().agn_oracle_replace(_pd(X.view(np.float64)), _pd(amp), int(n),
                                    _pd(Y.view(np.float64))), "replace")
    return Y


def argsort(y):
    y = _f64(y)
    perm = np.empty(len(y), dtype=np.uint32)
    _chk(_load().agn_oracle_argsort(_pd(y), len(y), _pu32(perm)), "argsort")
    return perm


def iterate(amp, x0, iters, tol=-1.0):
    """Returns (x_out, delta[iters], iters_done, rank[n])."""
    amp, x0 = _f64(amp), _f64(x0)
    n = len(x0)
    x = np.full(n, np.nan, dtype=np.float64)
    delta = np.zeros(max(iters, 1), dtype=np.float64)
    done = C.c_int32(0)
    rank = np.empty(n, dtype=np.uint32)
    _chk(_load().agn_oracle_iterate(_pd(amp), _pd(x0), n, int(iters), float(tol), _pd(x),
                                    _pd(delta), C.byref(done), _pu32(rank)), "iterate")
    return x, delta[:iters], int(done.value), rank


def generate(params: PsdParams, erdf, dt, iters, seed, curve_id=0, tol=-1.0):
    """Returns (x_out, delta[iters], iters_done, rank[n])."""
    erdf = _f64(erdf)
    n = len(erdf)
    x = np.full(n, np.nan, dtype=np.float64)
    delta = np.zeros(max(iters, 1), dtype=np.float64)
    done = C.c_int32(0)
    rank = np.empty(n, dtype=np.uint32)
    _chk(_load().agn_oracle_generate(C.byref(params), _pd(erdf), n, float(dt), int(iters),
                                     float(tol), int(seed), int(curve_id), _pd(x), _pd(delta),
                                     C.byref(done), _pu32(rank)), "generate")
    return x, delta[:iters], int(done.value), rank


def erdf_bpl(params: ErdfParams, n, seed, curve_id=0):
    out = np.full(n, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_erdf_bpl(C.byref(params), int(n), int(seed), int(curve_id), _pd(out)),
         "erdf_bpl")
    return out


def pdf_draw(params: PdfParams, n, seed, curve_id=0):
    """Draws 0..n-1 of the general PDF (lambda values)."""
    out = np.full(n, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_pdf_draw(C.byref(params), int(n), int(seed), int(curve_id), _pd(out)),
         "pdf_draw")
    return out


def pdf_draw_at(params: PdfParams, idx, seed, curve_id=0):
    """Draws #idx[i] of the general PDF (lambda values)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.full(len(idx), np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_pdf_draw_at(C.byref(params), int(seed), int(curve_id),
                                        idx.ctypes.data_as(C.POINTER(C.c_int64)), len(idx), _pd(out)),
         "pdf_draw_at")
    return out


def lag_stats(x, lags, units=0, dm_ref=(), lam_cut=0.0):
    """(sf2[K], exceed[K, J], pairs[K]) of one series: Eq. A6 structure function
    of x (units 0) or of -2.5 log10 x (units 1), and counts of pairs with
    |dm| above each threshold (Fig. 16), with an optional detection cut (Fig. 17)."""
    x = _f64(x)
    lags = np.ascontiguousarray(lags, dtype=np.int64)
    dm = np.ascontiguousarray(dm_ref, dtype=np.float64)
    K, J = len(lags), len(dm)
    sf2 = np.full(K, np.nan)
    exceed = np.zeros((K, max(J, 1)), dtype=np.uint64)
    pairs = np.zeros(K, dtype=np.uint64)
    pu64 = C.POINTER(C.c_uint64)
    _chk(_load().agn_oracle_lag_stats(_pd(x), len(x), lags.ctypes.data_as(C.POINTER(C.c_int64)), K, int(units),
                                      _pd(dm) if J else None, J, float(lam_cut), _pd(sf2),
                                      exceed.ctypes.data_as(pu64), pairs.ctypes.data_as(pu64)), "lag_stats")
    return sf2, exceed[:, :J], pairs


def uniform_chain(seed, stream, curve, chain, k):
    return _load().agn_oracle_uniform_chain(int(seed), int(stream), int(curve), int(chain), int(k))


def pdf_slice(params: PdfParams, n, n_chains, burn, seed, curve_id=0):
    """n slice-sampling draws (lambda values), chains interleaved."""
    out = np.full(n, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_pdf_slice(C.byref(params), int(n), int(n_chains), int(burn), int(seed),
                                      int(curve_id), _pd(out)), "pdf_slice")
    return out


def periodogram(x):
    x = _f64(x)
    P = np.full(len(x) // 2 + 1, np.nan, dtype=np.float64)
    _chk(_load().agn_oracle_periodogram(_pd(x), len(x), _pd(P)), "periodogram")
    return P


def psd_fit(f, pbar, f_br, a_low0=1.0, a_high0=2.0):
    """Eq. 3 fitted to a binned periodogram in log10 space with the break held
    at f_br: returns (log10 A, a_low, a_high, rms of the log10 residuals)."""
    f, pbar = _f64(f), _f64(pbar)
    out = np.full(4, np.nan)
    _chk(_load().agn_oracle_psd_fit(_pd(f), _pd(pbar), len(f), float(f_br), float(a_low0), float(a_high0),
                                    _pd(out)), "psd_fit")
    return out


def log_binned_mean_f(P, n, dt, dex=0.1):
    """The log bins of log_binned, with each bin's frequency the arithmetic mean
    of the f_j it holds.  Returns (f_mean, mean P)."""
    j = np.arange(1, n // 2 + 1)
    f = j / (n * dt)
    b = np.floor(np.log10(f / f[0]) / dex + 1e-9).astype(np.int64)
    nb = int(b.max()) + 1
    s = np.bincount(b, weights=P[1:], minlength=nb)
    sf = np.bincount(b, weights=f, minlength=nb)
    c = np.bincount(b, minlength=nb)
    keep = c > 0
    return sf[keep] / c[keep], s[keep] / c[keep]


def log_binned(P, n, dt, dex=0.1):
    """Log-binned periodogram: bins of `dex` in log10 f starting at f_1 (j >= 1),
    arithmetic mean of P_j per bin, empty bins dropped.  Returns (f_center, mean)."""
    j = np.arange(1, n // 2 + 1)
    f = j / (n * dt)
    b = np.floor(np.log10(f / f[0]) / dex + 1e-9).astype(np.int64)
    nb = int(b.max()) + 1
    s = np.bincount(b, weights=P[1:], minlength=nb)
    c = np.bincount(b, minlength=nb)
    keep = c > 0
    fc = f[0] * 10.0 ** ((np.arange(nb) + 0.5) * dex)
    return fc[keep], s[keep] / c[keep]
