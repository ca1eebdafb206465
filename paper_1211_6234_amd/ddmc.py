"""Python binding of the C ABI in ``include/ddmc.h`` (argument marshalling only).

Every function forwards to the same-named entry point of ``libddmc.so``;
PyTorch supplies device memory (tensors) and streams.  Nothing here computes:
there is no CPU fallback, and importing this module fails loudly when the
library has not been built (``python -m paper_1211_6234_amd.build``).

Array conventions (see the header): spins and fields are device tensors of
shape [R, 3, L, L] (float64 for a DDMC_F64 plan, float32 for DDMC_F32);
the kernel W64 is float64 [4, L, L]; replica parameters live on the device as
a uint8 tensor of R * 56 bytes produced by ``replica_params_upload``.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddmc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ddmc.h")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP = range(5)
F64, F32 = 0, 1
FIELD_AUTO, FIELD_DIRECT, FIELD_FFT, FIELD_FFT_LDS = 0, 1, 2, 3
MULTI_MAX_GROUPS = 8
NOBS = 26
KERNELS = ("direct_field", "update", "fft_columns", "fft_rows_sweep", "fft_rows", "observables",
           "fft_rows_sample")
OBS = dict(E=0, EEX=1, EDIP=2, EANI=3, MX=4, MY=5, MZ=6, MABS=7, MPAR=8, MZABS=9,
           NH=10, NV=13, ORIENT=16, WALLDENS=19, Q=20, ETASUM=21, MSTH=22, MSTV=23, ETAS=24, NONFINITE=25)
HEISENBERG, ISING = 0, 1
M_ALL = -1          # lattice_sum_kernel: every periodic image
PARAMS_BYTES = 56


class DDMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ddmc status %d: %s" % (status, msg))
        self.status = status


class ReplicaParams(C.Structure):
    _fields_ = [("T", C.c_double), ("J", C.c_double), ("K2", C.c_double), ("K4", C.c_double),
                ("g", C.c_double), ("seed", C.c_uint64), ("replica_id", C.c_uint32),
                ("model", C.c_uint32)]


assert C.sizeof(ReplicaParams) == PARAMS_BYTES

_lib = None


def lib():
    """Load libddmc.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libddmc.so is not built: run python -m paper_1211_6234_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
        st = C.c_int
        L.lattice_sum_kernel.argtypes = [i32, i32, vp, vp]
        L.ddmc_plan_create.argtypes = [i32, i32, i32, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.ddmc_plan_destroy.argtypes = [vp]
        L.ddmc_plan_algo.argtypes = [vp, C.POINTER(C.c_int)]
        L.ddmc_plan_device_bytes.argtypes = [i32, i32, C.c_int, C.c_int, C.POINTER(C.c_uint64)]
        L.replica_params_upload.argtypes = [i32, vp, vp, vp]
        L.local_field.argtypes = [vp, i32, vp, vp, i32, vp]
        L.init_spins.argtypes = [vp, i32, vp, vp, vp]
        L.metropolis_sweep.argtypes = [vp, i32, vp, vp, u64, i32, vp, vp]
        L.metropolis_sweep_dev.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp]
        L.metropolis_sweep_multi.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp, vp]
        L.metropolis_sample.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, vp]
        L.trial_energies.argtypes = [vp, i32, vp, vp, vp, u32, i32, vp, vp, vp, vp]
        L.metropolis_sweep_coset.argtypes = [vp, i32, vp, vp, i32, vp, i32, vp, vp]
        L.coset_error_bound.argtypes = [i32, i32, i32, C.POINTER(C.c_double)]
        L.parallel_tempering_swap.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp]
        L.observables.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.spins_convert.argtypes = [i32, i32, vp, C.c_int, vp, C.c_int, vp]
        L.observables_noalloc.argtypes = [i32, C.c_int, i32, vp, vp, vp, vp, vp, vp]
        L.ddmc_plan_profile.argtypes = [vp, i32]
        L.ddmc_plan_profile_read.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.ddmc_last_error.argtypes = []
        L.ddmc_last_error.restype = C.c_char_p
        for name in ("lattice_sum_kernel", "ddmc_plan_create", "ddmc_plan_destroy", "ddmc_plan_algo",
                     "ddmc_plan_device_bytes",
                     "replica_params_upload", "local_field", "init_spins", "metropolis_sweep", "metropolis_sweep_dev",
                     "metropolis_sweep_multi",
                     "metropolis_sample", "metropolis_sweep_coset", "coset_error_bound",
                     "parallel_tempering_swap", "trial_energies", "observables", "ddmc_plan_profile", "ddmc_plan_profile_read",
                     "spins_convert", "observables_noalloc"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/ddmc.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def _check(status):
    if status != OK:
        raise DDMCError(status, lib().ddmc_last_error().decode())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t, dtype=None, numel=None, what="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (what, t.numel(), numel))
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------- calls
def lattice_sum_kernel(L, M, W64=None, stream=None):
    """FP64 lattice-summed dipole tensor, returned as a [4, L, L] device tensor."""
    if W64 is None:
        W64 = torch.empty((4, L, L), dtype=torch.float64, device="cuda")
    _check(lib().lattice_sum_kernel(L, M, _ptr(W64, torch.float64, 4 * L * L, "W64"), _stream(stream)))
    return W64


_ALGO = {"auto": FIELD_AUTO, "direct": FIELD_DIRECT, "fft": FIELD_FFT, "fft_lds": FIELD_FFT_LDS}


def plan_device_bytes(L, R_max, prec="f32", algo="auto"):
    """Device bytes a Plan(L, M, R_max, prec, algo) allocates and keeps."""
    b = C.c_uint64()
    _check(lib().ddmc_plan_device_bytes(int(L), int(R_max), {"f64": F64, "f32": F32}[prec],
                                        _ALGO[algo],
                                        C.byref(b)))
    return b.value


class Plan:
    """Owns a ddmc_plan (derived kernel forms + workspace for R_max replicas)."""

    def __init__(self, L, M, R_max, prec="f32", algo="auto", W64=None, stream=None):
        self.L, self.M, self.R_max = int(L), int(M), int(R_max)
        self.prec = {"f64": F64, "f32": F32}[prec]
        self.dtype = torch.float64 if self.prec == F64 else torch.float32
        a = _ALGO[algo]
        if W64 is None:
            W64 = lattice_sum_kernel(L, M, stream=stream)
            # plan creation reads W64 on the null stream: wait for the stream it was written on
            if isinstance(stream, torch.cuda.Stream):
                stream.synchronize()
            elif stream is None:
                torch.cuda.current_stream().synchronize()
            else:
                torch.cuda.synchronize()
        self.W64 = W64
        h = C.c_void_p()
        _check(lib().ddmc_plan_create(self.L, self.M, self.R_max, self.prec, a,
                                      _ptr(W64, torch.float64, 4 * L * L, "W64"), C.byref(h)))
        self._h = h
        # held by the plan so that destruction at interpreter exit does not
        # depend on module globals that may already be cleared
        self._destroy = lib().ddmc_plan_destroy
        v = C.c_int()
        _check(lib().ddmc_plan_algo(h, C.byref(v)))
        self.algo = {FIELD_DIRECT: "direct", FIELD_FFT: "fft", FIELD_FFT_LDS: "fft_lds"}[v.value]

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._h = None
            self._destroy(h)

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def profile(self, enable=True):
        """Turn the plan's event-based kernel timing on (clearing totals) or off."""
        _check(lib().ddmc_plan_profile(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since profiling was enabled (synchronizes)."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n = C.c_double(), C.c_int64()
            _check(lib().ddmc_plan_profile_read(self.handle, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def spins(self, R):
        return torch.empty((R, 3, self.L, self.L), dtype=self.dtype, device="cuda")


def pack_params(replicas):
    """Host bytes of R parameter records (dicts with T, J, K2, K4, g, seed,
    replica_id and model: HEISENBERG (default) or ISING)."""
    arr = (ReplicaParams * len(replicas))()
    for k, p in enumerate(replicas):
        arr[k] = ReplicaParams(float(p["T"]), float(p.get("J", 1.0)), float(p.get("K2", 0.0)),
                               float(p.get("K4", 0.0)), float(p.get("g", 0.0)), int(p.get("seed", 0)),
                               int(p.get("replica_id", k)), int(p.get("model", HEISENBERG)))
    return arr


def replica_params_upload(replicas, dev=None, stream=None):
    """Validate and copy parameter records to the device; returns the uint8 device tensor."""
    R = len(replicas)
    host = pack_params(replicas)
    if dev is None:
        dev = torch.empty(max(1, R) * PARAMS_BYTES, dtype=torch.uint8, device="cuda")
    _check(lib().replica_params_upload(R, C.cast(host, C.c_void_p),
                                       _ptr(dev, torch.uint8, R * PARAMS_BYTES, "params"), _stream(stream)))
    return dev


def _n(plan, R, comps=3):
    return R * comps * plan.L * plan.L


def local_field(plan, R, s, h, color=-1, stream=None):
    _check(lib().local_field(plan.handle, R, _ptr(s, plan.dtype, _n(plan, R), "s"),
                             _ptr(h, plan.dtype, _n(plan, R), "h"), color, _stream(stream)))


def init_spins(plan, R, params, s, stream=None):
    _check(lib().init_spins(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                            _ptr(s, plan.dtype, _n(plan, R), "s"), _stream(stream)))


def metropolis_sweep(plan, R, params, s, sweep0, nsweeps, accepted=None, stream=None):
    _check(lib().metropolis_sweep(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                  _ptr(s, plan.dtype, _n(plan, R), "s"), int(sweep0), int(nsweeps),
                                  _ptr(accepted, torch.int64, R, "accepted"), _stream(stream)))


def metropolis_sweep_dev(plan, R, params, s, counter, nsweeps, accepted=None, stream=None):
    """Sweeps whose first index per replica is read from (and advanced in) the
    device int64 tensor `counter` of R entries."""
    _check(lib().metropolis_sweep_dev(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                      _ptr(s, plan.dtype, _n(plan, R), "s"), _ptr(counter, torch.int64, R, "counter"),
                                      int(nsweeps), _ptr(accepted, torch.int64, R, "accepted"), _stream(stream)))


def metropolis_sweep_multi(groups, nsweeps, stream=None):
    """metropolis_sweep_dev for several plans (lattice sizes) in one launch.
    groups: list of (plan, R, params, s, counter, accepted or None)."""
    n = len(groups)
    P = C.c_void_p * n
    plans = P(*[g[0].handle for g in groups])
    Rs = (C.c_int32 * n)(*[int(g[1]) for g in groups])
    prm = P(*[_ptr(g[2], torch.uint8, g[1] * PARAMS_BYTES, "params") for g in groups])
    ss = P(*[_ptr(g[3], g[0].dtype, _n(g[0], g[1]), "s") for g in groups])
    ctr = P(*[_ptr(g[4], torch.int64, g[1], "counter") for g in groups])
    have_acc = any(g[5] is not None for g in groups)
    acc = P(*[_ptr(g[5], torch.int64, g[1], "accepted") for g in groups]) if have_acc else None
    _check(lib().metropolis_sweep_multi(n, plans, Rs, prm, ss, ctr, int(nsweeps), acc, _stream(stream)))


def metropolis_sample(plan, R, params, s, counter, nsweeps, obs, eta_acc=None, accepted=None, stream=None):
    """nsweeps sweeps (as metropolis_sweep_dev) with one observables sample
    after each: obs is a device float64 tensor of nsweeps * R * NOBS."""
    _check(lib().metropolis_sample(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                   _ptr(s, plan.dtype, _n(plan, R), "s"), _ptr(counter, torch.int64, R, "counter"),
                                   int(nsweeps), _ptr(obs, torch.float64, max(0, int(nsweeps)) * R * NOBS, "obs"),
                                   _ptr(eta_acc, torch.float64, _n(plan, R, 1), "eta_acc"),
                                   _ptr(accepted, torch.int64, R, "accepted"), _stream(stream)))


def metropolis_sweep_coset(plan, R, params, s, l, counter, nsweeps, accepted=None, stream=None):
    """Sweeps of the l-coset simultaneous update (Sec. 3.1)."""
    _check(lib().metropolis_sweep_coset(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                        _ptr(s, plan.dtype, _n(plan, R), "s"), int(l),
                                        _ptr(counter, torch.int64, R, "counter"), int(nsweeps),
                                        _ptr(accepted, torch.int64, R, "accepted"), _stream(stream)))


def parallel_tempering_swap(plan, R, params, s, obs, counter, parity, swaps=None, stream=None):
    """Replica exchange between ladder neighbours (r, r + 1), r = parity mod 2;
    obs: device float64 [R][NOBS] with energies of the current states."""
    _check(lib().parallel_tempering_swap(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                         _ptr(s, plan.dtype, _n(plan, R), "s"),
                                         _ptr(obs, torch.float64, R * NOBS, "obs"),
                                         _ptr(counter, torch.int64, R, "counter"), int(parity),
                                         _ptr(swaps, torch.int64, R, "swaps"), _stream(stream)))


def coset_error_bound(L, l, all_images=False):
    """eq. (10) bound (units of C_D) for the l-coset update."""
    eps = C.c_double()
    _check(lib().coset_error_bound(int(L), int(l), 1 if all_images else 0, C.byref(eps)))
    return eps.value


def trial_energies(plan, R, params, s, h, sweep, color, dE, u, S=None, stream=None):
    _check(lib().trial_energies(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                _ptr(s, plan.dtype, _n(plan, R), "s"), _ptr(h, plan.dtype, _n(plan, R), "h"),
                                int(sweep), int(color), _ptr(dE, plan.dtype, _n(plan, R, 1), "dE"),
                                _ptr(u, plan.dtype, _n(plan, R, 1), "u"),
                                _ptr(S, plan.dtype, _n(plan, R), "S"), _stream(stream)))


def spins_convert(R, L, src, dst, stream=None):
    """Copy R states between precisions (the dtypes of the two tensors decide)."""
    prec = {torch.float64: F64, torch.float32: F32}
    n = R * 3 * L * L
    _check(lib().spins_convert(R, L, _ptr(src, None, n, "src"), prec[src.dtype], _ptr(dst, None, n, "dst"),
                               prec[dst.dtype], _stream(stream)))


def observables(plan, R, params, s, h, out, eta_acc=None, stream=None):
    _check(lib().observables(plan.handle, R, _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                             _ptr(s, plan.dtype, _n(plan, R), "s"),
                             _ptr(h, plan.dtype, _n(plan, R), "h"),
                             _ptr(out, torch.float64, R * NOBS, "out"),
                             _ptr(eta_acc, torch.float64, _n(plan, R, 1), "eta_acc"), _stream(stream)))


NOALLOC_R_MAX = 256


def observables_noalloc(L, R, params, s, h, out, eta_acc=None, stream=None):
    """`observables` without a plan or any allocation (static scratch of
    NOALLOC_R_MAX replicas); the precision is that of s."""
    prec = {torch.float64: F64, torch.float32: F32}[s.dtype]
    n = R * 3 * L * L
    _check(lib().observables_noalloc(int(L), prec, int(R), _ptr(params, torch.uint8, R * PARAMS_BYTES, "params"),
                                     _ptr(s, s.dtype, n, "s"), _ptr(h, s.dtype, n, "h"),
                                     _ptr(out, torch.float64, R * NOBS, "out"),
                                     _ptr(eta_acc, torch.float64, R * L * L, "eta_acc"), _stream(stream)))
