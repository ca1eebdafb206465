"""FP64 CPU oracle for the dipolar Heisenberg Monte Carlo hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  It wraps the plain C
reference in ``oracle.c`` (built with gcc, never with the HIP toolchain) and
shares no code with the HIP library.

Every array is float64, spins component-major ``s[3][N]`` with site
``i = y*L + x``; the dipole kernel is ``W[4][L][L]`` with planes xx, yy, xy,
zz.  See ``oracle.c`` for the equations followed and the readings taken.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

# observable slots (mirrors the enum in oracle.h)
OBS = dict(E=0, EEX=1, EDIP=2, EANI=3, MX=4, MY=5, MZ=6, MABS=7, MPAR=8, MZABS=9,
           NH=10, NV=13, ORIENT=16, WALLDENS=19, Q=20, ETASUM=21, MSTH=22, MSTV=23, ETAS=24, NONFINITE=25)
NOBS = 26


class Params(C.Structure):
    _fields_ = [("T", C.c_double), ("J", C.c_double), ("K2", C.c_double),
                ("K4", C.c_double), ("g", C.c_double), ("seed", C.c_uint64),
                ("replica_id", C.c_uint32), ("model", C.c_uint32)]


def params(T, J=1.0, K2=0.0, K4=0.0, g=0.0, seed=0, replica_id=0, model=0):
    """model 0: Heisenberg (uniform trial directions); 1: Ising (trial = reversal)."""
    return Params(float(T), float(J), float(K2), float(K4), float(g), int(seed),
                  int(replica_id), int(model))


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, IEEE arithmetic)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB points the pins at another build of oracle.c (the
        # mutation test plants mistakes in copies and expects the pins to fail)
        path = os.environ.get("ORACLE_LIB")
        if not path:
            build()
            path = _SO
        L = C.CDLL(path)
        P = C.POINTER
        d, u32, u64, i32, lng = C.c_double, C.c_uint32, C.c_uint64, C.c_int, C.c_long
        vp = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_u01.argtypes = [u32]
        L.orc_u01.restype = d
        L.orc_draw.argtypes = [u64, u32, u32, u32, u32, P(d)]
        L.orc_direction.argtypes = [d, d, P(d)]
        L.orc_lattice_sum_kernel.argtypes = [i32, i32, vp]
        L.orc_lattice_sum_ewald.argtypes = [i32, d, vp]
        L.orc_field_site.argtypes = [i32, vp, vp, lng, P(d)]
        L.orc_field.argtypes = [i32, vp, vp, vp]
        L.orc_field_images.argtypes = [i32, i32, vp, vp]
        L.orc_energy.argtypes = [i32, vp, P(Params), vp, P(d)]
        L.orc_delta_e.argtypes = [i32, vp, P(Params), vp, vp, lng, P(d)]
        L.orc_delta_e.restype = d
        L.orc_metropolis_accept.argtypes = [d, d, d]
        L.orc_metropolis_accept.restype = i32
        L.orc_init_spins.argtypes = [i32, u64, u32, vp]
        L.orc_init_ising.argtypes = [i32, u64, u32, vp]
        L.orc_sweep_sequential.argtypes = [i32, vp, P(Params), vp, vp, u32, i32, P(u64)]
        L.orc_trial_energies.argtypes = [i32, vp, P(Params), vp, vp, u32, i32, vp, vp, vp]
        L.orc_sweep_checkerboard.argtypes = [i32, vp, P(Params), vp, u32, i32, P(u64)]
        L.orc_observables.argtypes = [i32, vp, P(Params), vp, vp, vp]
        L.orc_variances.argtypes = [i32, vp, P(d)]
        L.orc_staggered_susceptibility.argtypes = [i32, d, i32, vp]
        L.orc_staggered_susceptibility.restype = d
        L.orc_sweep_coset.argtypes = [i32, vp, P(Params), vp, i32, u32, i32, P(u64)]
        L.orc_coset_error.argtypes = [i32, i32, i32]
        L.orc_coset_error.restype = d
        L.orc_pt_swap.argtypes = [i32, i32, P(Params), vp, vp, vp, i32, vp]
        L.orc_run.argtypes = [i32, i32, P(Params), vp, u32, i32, i32, i32, i32, vp, i32, vp,
                              P(u64)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------- Philox
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def draw(seed, replica, sweep, site, purpose):
    u = (C.c_double * 4)()
    lib().orc_draw(seed, replica, sweep, site, purpose, u)
    return np.array(u[:])


def direction(u0, u1):
    S = (C.c_double * 3)()
    lib().orc_direction(u0, u1, S)
    return np.array(S[:])


# ---------------------------------------------------------------- kernel and field
def lattice_sum_kernel(L, M):
    W = np.zeros((4, L, L))
    lib().orc_lattice_sum_kernel(L, M, _ptr(W))
    return W


def lattice_sum_ewald(L, eta=None):
    """All images (Ewald-Harris split); eta defaults to L / 4."""
    W = np.zeros((4, L, L))
    lib().orc_lattice_sum_ewald(L, float(L / 4.0 if eta is None else eta), _ptr(W))
    return W


def field(L, W, s):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L))
    h = np.zeros((3, L * L))
    lib().orc_field(L, _ptr(W), _ptr(s), _ptr(h))
    return h


def field_site(L, W, s, i):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L))
    h = (C.c_double * 3)()
    lib().orc_field_site(L, _ptr(W), _ptr(s), int(i), h)
    return np.array(h[:])


def field_images(L, M, s):
    s = _f64(s, (3, L * L))
    h = np.zeros((3, L * L))
    lib().orc_field_images(L, M, _ptr(s), _ptr(h))
    return h


# ---------------------------------------------------------------- energy and moves
def energy(L, W, p, s):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L))
    parts = (C.c_double * 4)()
    lib().orc_energy(L, _ptr(W), C.byref(p), _ptr(s), parts)
    return dict(ex=parts[0], dip=parts[1], ani=parts[2], total=parts[3])


def delta_e(L, W, p, s, h, k, S):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L)); h = _f64(h, (3, L * L))
    Sa = (C.c_double * 3)(*[float(v) for v in S])
    return lib().orc_delta_e(L, _ptr(W), C.byref(p), _ptr(s), _ptr(h), int(k), Sa)


def metropolis_accept(dE, T, u):
    return bool(lib().orc_metropolis_accept(dE, T, u))


def init_spins(L, seed, replica):
    s = np.zeros((3, L * L))
    lib().orc_init_spins(L, seed, replica, _ptr(s))
    return s


def init_ising(L, seed, replica):
    s = np.zeros((3, L * L))
    lib().orc_init_ising(L, seed, replica, _ptr(s))
    return s


def sweep_sequential(L, W, p, s, h, sweep0, nsweeps):
    """Runs in place on copies; returns (s, h, accepted)."""
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L)).copy(); h = _f64(h, (3, L * L)).copy()
    acc = C.c_uint64(0)
    lib().orc_sweep_sequential(L, _ptr(W), C.byref(p), _ptr(s), _ptr(h), sweep0, nsweeps,
                               C.byref(acc))
    return s, h, acc.value


def trial_energies(L, W, p, s, h, sweep, color):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L)); h = _f64(h, (3, L * L))
    N = L * L
    dE = np.zeros(N); u2 = np.zeros(N); S = np.zeros((3, N))
    lib().orc_trial_energies(L, _ptr(W), C.byref(p), _ptr(s), _ptr(h), sweep, color,
                             _ptr(dE), _ptr(u2), _ptr(S))
    return dE, u2, S


def sweep_checkerboard(L, W, p, s, sweep0, nsweeps):
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L)).copy()
    acc = C.c_uint64(0)
    lib().orc_sweep_checkerboard(L, _ptr(W), C.byref(p), _ptr(s), sweep0, nsweeps,
                                 C.byref(acc))
    return s, acc.value


def sweep_coset(L, W, p, s, l, sweep0, nsweeps):
    """l-coset simultaneous updates (Sec. 3.1); returns (s, accepted)."""
    W = _f64(W, (4, L, L)); s = _f64(s, (3, L * L)).copy()
    acc = C.c_uint64(0)
    lib().orc_sweep_coset(L, _ptr(W), C.byref(p), _ptr(s), int(l), sweep0, nsweeps, C.byref(acc))
    return s, acc.value


def coset_error(L, l, all_images=False):
    """Eq. (10) error bound for the coset update, C_D = 1."""
    return lib().orc_coset_error(L, l, 1 if all_images else 0)


def pt_swap(L, plist, s, E, rounds, parity, swaps=None):
    """Replica exchange between ladder neighbours; s [R][3][N] and swaps [R]
    (uint64) updated in place."""
    R = len(plist)
    arr = (Params * R)(*plist)
    E = np.ascontiguousarray(E, dtype=np.float64)
    rd = np.ascontiguousarray(rounds, dtype=np.uint32)
    assert s.dtype == np.float64 and s.flags.c_contiguous and s.shape == (R, 3, L * L)
    if swaps is not None:
        assert swaps.dtype == np.uint64 and swaps.shape == (R,)
    lib().orc_pt_swap(L, R, arr, _ptr(s), _ptr(E), _ptr(rd), int(parity), _ptr(swaps))


def observables(L, W, p, s, eta_acc=None):
    """W may be None (energy slots then NaN).  eta_acc is updated in place."""
    s = _f64(s, (3, L * L))
    if W is not None:
        W = _f64(W, (4, L, L))
    out = np.zeros(NOBS)
    lib().orc_observables(L, _ptr(W), C.byref(p), _ptr(s), _ptr(out), _ptr(eta_acc))
    return out


def variances(obs):
    """eq. (18) over the rows of obs [nsamp][NOBS] (or more columns: only the
    first NOBS are read): (sigma^2(M_par), sigma^2(O_z), sigma^2(eta))."""
    obs = np.ascontiguousarray(np.asarray(obs, dtype=np.float64)[:, :NOBS])
    assert obs.shape[1] == NOBS and obs.shape[0] > 0
    out = (C.c_double * 3)()
    lib().orc_variances(int(obs.shape[0]), _ptr(obs), out)
    return np.array(out[:])


def staggered_susceptibility(L, T, obs):
    """chi_st = (L^2 / T)(<m_st^2> - <m_st>^2) over the rows of obs [nsamp][NOBS]."""
    obs = np.ascontiguousarray(np.asarray(obs, dtype=np.float64)[:, :NOBS])
    assert obs.shape[1] == NOBS and obs.shape[0] > 0
    return lib().orc_staggered_susceptibility(int(L), float(T), int(obs.shape[0]), _ptr(obs))


def run(L, M, p, s, sweep0, nburn, nsamp, mode="sequential", with_energy=False, nbatch=0):
    """Burn-in then one sample per sweep.  Returns dict(obs, eta_acc, s, accepted)."""
    s = _f64(s, (3, L * L)).copy()
    obs = np.zeros((nsamp, NOBS))
    eta = np.zeros((nbatch, L * L)) if nbatch > 0 else None
    acc = C.c_uint64(0)
    lib().orc_run(L, M, C.byref(p), _ptr(s), sweep0, nburn, nsamp,
                  0 if mode == "sequential" else 1, 1 if with_energy else 0, _ptr(obs),
                  nbatch, _ptr(eta), C.byref(acc))
    return dict(obs=obs, eta_acc=eta, s=s, accepted=acc.value)
