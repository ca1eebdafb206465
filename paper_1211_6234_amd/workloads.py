"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws inputs (spin configurations, replica parameter sets);
it holds none of the method's arithmetic, and it is the only code that both
the HIP path's callers and the FP64 oracle's callers use.

The paper runs no public dataset: its workload is a parameter set (Sec. 4.1:
L = 64, J/C_D = 8.9, K/C_D = 15, a in {-1, 0, 2}, T/C_D in [0.2, 10]).  The
recipes below are the five synthetic workloads this project measures, in
exchange units (J = 1, g = C_D / J), with the anisotropy written as
-K2 sz^2 - K4 sz^4.
"""
from __future__ import annotations

import numpy as np


def random_spins(N: int, R: int, seed: int) -> np.ndarray:
    """R independent states of N unit vectors, isotropic, as float64 [R][3][N]."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(R, 3, N))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def replica(T, J=1.0, K2=0.0, K4=0.0, g=0.0, seed=0, replica_id=0, model=0) -> dict:
    """One replica's parameters; model 0 Heisenberg, 1 Ising."""
    return dict(T=float(T), J=float(J), K2=float(K2), K4=float(K4), g=float(g),
                seed=int(seed), replica_id=int(replica_id), model=int(model))


# ----------------------------------------------------------------- workloads
def cpu_sized():
    """L = 16, one replica: g = 0.1, K2 = 1, K4 = 0, T = 0.7, images |a|,|b| <= 8,
    seed 0, 2000 sequential sweeps in FP64."""
    return dict(name="L16_single_fp64", L=16, M=8, sweeps=2000,
                replicas=[replica(0.7, 1.0, 1.0, 0.0, 0.1, seed=0, replica_id=0)])


def checkerboard_l64(T: float, seed: int):
    """L = 64, one replica: g = 0.1, K2 = 1.5, K4 = -0.5, T in {0.5, 0.8}."""
    return dict(name="L64_T%.2f_seed%d" % (T, seed), L=64, M=8, sweeps=10000,
                replicas=[replica(T, 1.0, 1.5, -0.5, 0.1, seed=seed, replica_id=0)])


def ladder_l128(R: int = 32, K4: float = 0.0):
    """Temperature ladder: L = 128, R replicas with T linearly spaced over
    [0.3, 1.2], g = 0.15, K2 = 2.0, K4 in {-1, 0, +1}; replica r has seed 1000 + r."""
    Ts = np.linspace(0.3, 1.2, R) if R > 1 else np.array([0.3])
    return dict(name="L128_R%d_ladder_K4%+g" % (R, K4), L=128, M=8, sweeps=5000,
                replicas=[replica(T, 1.0, 2.0, K4, 0.15, seed=1000 + r, replica_id=r)
                          for r, T in enumerate(Ts)])


def ladder_l32_pt(R: int = 32):
    """A replica-exchange ladder whose neighbours do exchange: L = 32
    (N = 1024), R replicas with T linearly spaced over [0.6, 1.2]
    (dT ~ 0.02, so that dBeta dE is of order one), g = 0.15, K2 = 2.0,
    K4 = 0; replica r has seed 3000 + r."""
    Ts = np.linspace(0.6, 1.2, R) if R > 1 else np.array([0.6])
    return dict(name="L32_R%d_pt_ladder" % R, L=32, M=8, sweeps=2000,
                replicas=[replica(T, 1.0, 2.0, 0.0, 0.15, seed=3000 + r, replica_id=r)
                          for r, T in enumerate(Ts)])


def large_l256(R: int = 64):
    """L = 256, R replicas: g = 0.2, K2 = 2.5, K4 = -0.8, T ~ U[0.4, 1.0]
    (numpy seed 5); replica r has Philox seed 2000 + r."""
    rng = np.random.default_rng(5)
    Ts = rng.uniform(0.4, 1.0, size=R)
    return dict(name="L256_R%d" % R, L=256, M=8, sweeps=2000,
                replicas=[replica(T, 1.0, 2.5, -0.8, 0.2, seed=2000 + r, replica_id=r)
                          for r, T in enumerate(Ts)])


def served_mix(n_requests: int, arrival_seed: int = 0, rate: float = 50.0):
    """Poisson arrivals (mean `rate` per second) of independent simulations:
    L ~ U{32, 48, 64, 96, 128}, T ~ U[0.3, 1.2], K2 ~ U[0.5, 2.5],
    K4 ~ U[-1, 1], g ~ U[0.05, 0.2], 2000 sweeps; request i has seed i."""
    rng = np.random.default_rng(arrival_seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    Ls = rng.choice([32, 48, 64, 96, 128], size=n_requests)
    out = []
    for i in range(n_requests):
        out.append(dict(arrival=float(t[i]), L=int(Ls[i]), M=8, sweeps=2000,
                        params=replica(rng.uniform(0.3, 1.2), 1.0, rng.uniform(0.5, 2.5),
                                       rng.uniform(-1, 1), rng.uniform(0.05, 0.2),
                                       seed=i, replica_id=0)))
    return out


def film_scan(temps, avals=(-1.0, 0.0, 2.0), Jd=8.9, Kd=15.0, seed0=3000, reading="double_dipole"):
    """The paper's own parameter set (Sec. 4.1): L = 64, J/C_D = 8.9,
    |K|/C_D = 15, a in {-1, 0, 2}, k_B T / C_D over `temps`, in this library's
    units (E = -J sum over bonds s_i.s_j + (g/2) sum_ij s_i W s_j - K2 s_z^2 -
    K4 s_z^4, J = 1).

    The stated ground-state stripe widths (w = 8 at J/C_D = 8.9, Sec. 4.1;
    w = 1 at J/C_D = 1.7, the Ising appendix) come out of the energy only when
    the pair dipole coupling is twice C_D relative to the bond exchange J:
    g = 2 / 8.9.  That fixes the ratio, not the scale of T and K (given in
    units of C_D):
      "double_dipole" (default): the bond exchange is the paper's J and the
        pair dipole coupling 2 C_D, so T = (k_B T / C_D) / 8.9 and
        |K| = 15 / 8.9.  This reading reproduces the points the paper prints
        (M_par ~ .46 near k_B T / C_D = 4.5 for a = 0, the sharp
        reorientation at 4 for a = 2, paramagnetic above about 8);
      "half_exchange": the bond exchange is J/2 with C_D as written, so
        T = (k_B T / C_D) g and |K| = 15 g (no in-plane phase appears).
    The anisotropy K((1 - a) s_z^2 + a s_z^4) with K = -|K| is written as
    K2 = (1 - a)|K|, K4 = a |K|.  Replica (a index, T index) has seed
    seed0 + index and replica id = index."""
    g = 2.0 / Jd
    unit = {"half_exchange": g, "double_dipole": 1.0 / Jd}[reading]   # C_D in units of the bond exchange
    Kabs = Kd * unit
    reps = []
    for ia, a in enumerate(avals):
        for it, Td in enumerate(temps):
            k = ia * len(temps) + it
            reps.append(dict(replica(Td * unit, 1.0, (1.0 - a) * Kabs, a * Kabs, g, seed=seed0 + k, replica_id=k),
                             a=float(a), T_CD=float(Td)))
    return dict(name="film_L64_J8.9_K15_%s" % reading, L=64, stripe_width=8, replicas=reps)


def striped_spins(L: int, w: int, R: int) -> np.ndarray:
    """R copies of the perpendicular striped state (Sec. 4.1 start): s = +z on
    columns x with floor(x / w) even, -z on the others; float64 [R][3][L*L]."""
    x = np.arange(L * L) % L
    sz = np.where((x // w) % 2 == 0, 1.0, -1.0)
    s = np.zeros((R, 3, L * L))
    s[:, 2, :] = sz
    return s
