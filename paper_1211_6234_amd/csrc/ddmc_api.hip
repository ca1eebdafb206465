// ddmc_api.hip -- the C ABI of include/ddmc.h: argument validation, plan
// construction and dispatch to the kernels.  No call throws across the ABI.
#include <math.h>

#include <algorithm>
#include <new>
#include <string>

#include "internal.hpp"

namespace ddmc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ddmc_status fail(ddmc_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

ddmc_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return DDMC_OK;
    return fail(DDMC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static hipEvent_t prof_event(const ddmc_plan *p)
{
    if (!p->prof_free.empty()) {
        hipEvent_t e = p->prof_free.back();
        p->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_drain(const ddmc_plan *p, size_t n)
{
    n = std::min(n, p->prof_pending.size());
    for (size_t k = 0; k < n; ++k) {
        ddmc_prof_pair &q = p->prof_pending[k];
        float ms = 0.0f;
        if (hipEventSynchronize(q.stop) == hipSuccess && hipEventElapsedTime(&ms, q.start, q.stop) == hipSuccess) {
            p->prof_ms[q.kernel] += ms;
            p->prof_n[q.kernel] += 1;
        }
        p->prof_free.push_back(q.start);
        p->prof_free.push_back(q.stop);
    }
    p->prof_pending.erase(p->prof_pending.begin(), p->prof_pending.begin() + n);
}

prof_scope::prof_scope(const ddmc_plan *plan, int k, hipStream_t s) : p(plan), kernel(k), st(s)
{
    if (p && p->prof) {
        start = prof_event(p);
        if (start && hipEventRecord(start, st) != hipSuccess) start = nullptr;
    }
}

prof_scope::~prof_scope()
{
    if (!start) return;
    hipEvent_t stop = prof_event(p);
    if (!stop || hipEventRecord(stop, st) != hipSuccess) {
        p->prof_free.push_back(start);
        return;
    }
    p->prof_pending.push_back(ddmc_prof_pair{start, stop, kernel});
    if (p->prof_pending.size() > 8192) prof_drain(p, 4096);
}

static size_t elem_size(ddmc_prec p) { return p == DDMC_F64 ? sizeof(double) : sizeof(float); }

static bool valid_plan(const ddmc_plan *p) { return p != nullptr && p->L >= 2; }

// Device bytes of the arrays every plan allocates (the FFT workspace comes
// on top, from fft_plan_bytes); ddmc_plan_create allocates exactly these.
struct plan_sizes {
    size_t W, h, obs, done, part;
    size_t total() const { return W + h + obs + done + part; }
};

static plan_sizes plan_sizes_of(int L, int R_max, ddmc_prec prec, ddmc_field_algo algo)
{
    const size_t N = (size_t)L * L, es = elem_size(prec);
    plan_sizes z;
    z.W = 4 * N * es;
    z.h = (size_t)R_max * 3 * N * es;
    z.obs = (size_t)R_max * OBS_MAX_BLOCKS * OBS_NACC * sizeof(double);
    z.done = (size_t)R_max * sizeof(unsigned int);
    z.part = algo == DDMC_FIELD_DIRECT ? direct_partial_elems(L, R_max, es) * es : 0;
    return z;
}

static ddmc_status check_R(const ddmc_plan *p, int32_t R)
{
    if (R < 0) return fail(DDMC_EINVAL, "R must be >= 0");
    if (R > p->R_max) return fail(DDMC_EINVAL, "R exceeds the plan's R_max");
    return DDMC_OK;
}

template <typename T>
static ddmc_status field_dispatch(ddmc_plan *p, int R, const T *s, T *h, int color, hipStream_t st)
{
    if (p->algo == DDMC_FIELD_FFT) return fft_field<T>(p, R, s, h, color, st);
    return direct_field<T>(p, R, s, h, color, st);
}

template <typename T>
static ddmc_status sweep_direct(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s,
                                uint64_t *sweep_ctr, uint64_t sweep0, int nsweeps, uint64_t *accepted,
                                hipStream_t st)
{
    T *h = reinterpret_cast<T *>(p->h_ws);
    for (int t = 0; t < nsweeps; ++t) {
        const uint32_t sweep = (uint32_t)(sweep0 + (uint64_t)t);
        for (int color = 0; color < 2; ++color) {
            ddmc_status e = direct_field<T>(p, R, s, h, color, st);
            if (e != DDMC_OK) return e;
            const int last = (t == nsweeps - 1) && color == 1;
            hipError_t he = launch_update<T>(p, R, params, s, h, color, sweep_ctr, sweep, accepted, last,
                                             (uint64_t)nsweeps, st);
            if (he != hipSuccess) return hip_check(he, "update launch");
        }
    }
    return DDMC_OK;
}

// The l-coset schedule on the direct path: the full field, then the update
// of one coset, l^2 times per sweep.
template <typename T>
static ddmc_status sweep_direct_coset(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, int l,
                                      uint64_t *sweep_ctr, int nsweeps, uint64_t *accepted, hipStream_t st)
{
    T *h = reinterpret_cast<T *>(p->h_ws);
    const int ncos = l * l;
    for (int t = 0; t < nsweeps; ++t) {
        for (int k = 0; k < ncos; ++k) {
            ddmc_status e = direct_field<T>(p, R, s, h, -1, st);
            if (e != DDMC_OK) return e;
            const int last = (t == nsweeps - 1) && k == ncos - 1;
            hipError_t he = launch_update<T>(p, R, params, s, h, k, sweep_ctr, (uint32_t)t, accepted, last,
                                             (uint64_t)nsweeps, st, l);
            if (he != hipSuccess) return hip_check(he, "update launch");
        }
    }
    return DDMC_OK;
}

// The direct path samples with the standalone kernels: one sweep, the full
// field, the observables.
template <typename T>
static ddmc_status sample_direct(ddmc_plan *p, int R, const ddmc_replica_params *params, T *s, uint64_t *sweep_ctr,
                                 int nsweeps, uint64_t *accepted, double *obs, double *eta_acc, hipStream_t st)
{
    T *h = reinterpret_cast<T *>(p->h_ws);
    for (int t = 0; t < nsweeps; ++t) {
        ddmc_status e = sweep_direct<T>(p, R, params, s, sweep_ctr, 0, 1, accepted, st);
        if (e == DDMC_OK) e = direct_field<T>(p, R, s, h, -1, st);
        if (e != DDMC_OK) return e;
        hipError_t he = launch_observables<T>(p, R, params, s, h, obs + (long)t * R * DDMC_NOBS, eta_acc, st);
        if (he != hipSuccess) return hip_check(he, "observables launch");
    }
    return DDMC_OK;
}

static ddmc_status sweep_dispatch(ddmc_plan *p, int R, const ddmc_replica_params *params, void *s,
                                  uint64_t *sweep_ctr, uint64_t sweep0, int nsweeps, uint64_t *accepted,
                                  double *obs, double *eta_acc, hipStream_t st)
{
    if (p->sweep_lds) {
        uint64_t *const ctrs[1] = {sweep_ctr};
        uint64_t *const accs[1] = {accepted};
        const int Rs[1] = {R};
        ddmc_plan *const plans[1] = {p};
        const ddmc_replica_params *const prm[1] = {params};
        if (p->prec == DDMC_F64) {
            double *const ss[1] = {(double *)s};
            return lds_sweep<double>(1, plans, Rs, prm, ss, sweep_ctr ? ctrs : nullptr, sweep0, nsweeps, accs, obs,
                                     eta_acc, st);
        }
        float *const ss[1] = {(float *)s};
        return lds_sweep<float>(1, plans, Rs, prm, ss, sweep_ctr ? ctrs : nullptr, sweep0, nsweeps, accs, obs, eta_acc,
                                st);
    }
    if (p->algo == DDMC_FIELD_FFT) {
        if (p->prec == DDMC_F64)
            return fft_sweep<double>(p, R, params, (double *)s, sweep_ctr, sweep0, nsweeps, accepted, obs, eta_acc,
                                     st);
        return fft_sweep<float>(p, R, params, (float *)s, sweep_ctr, sweep0, nsweeps, accepted, obs, eta_acc, st);
    }
    if (obs) {
        if (p->prec == DDMC_F64)
            return sample_direct<double>(p, R, params, (double *)s, sweep_ctr, nsweeps, accepted, obs, eta_acc, st);
        return sample_direct<float>(p, R, params, (float *)s, sweep_ctr, nsweeps, accepted, obs, eta_acc, st);
    }
    if (p->prec == DDMC_F64)
        return sweep_direct<double>(p, R, params, (double *)s, sweep_ctr, sweep0, nsweeps, accepted, st);
    return sweep_direct<float>(p, R, params, (float *)s, sweep_ctr, sweep0, nsweeps, accepted, st);
}

}  // namespace ddmc

using namespace ddmc;

extern "C" {

const char *ddmc_last_error(void) { return g_last_error.c_str(); }

ddmc_status lattice_sum_kernel(int32_t L, int32_t M, double *W64, void *stream)
{
    if (L < 1 || L > 4096) return fail(DDMC_EINVAL, "lattice_sum_kernel: L must be in [1, 4096]");
    if (M < -1 || M > 1024) return fail(DDMC_EINVAL, "lattice_sum_kernel: M must be -1 (all images) or in [0, 1024]");
    if (!W64) return fail(DDMC_EINVAL, "lattice_sum_kernel: W64 is NULL");
    return hip_check(launch_lattice_sum(L, M, W64, (hipStream_t)stream), "lattice_sum_kernel launch");
}

ddmc_status ddmc_plan_destroy(ddmc_plan *p)
{
    if (!p) return DDMC_OK;
    hipFree(p->W);
    hipFree(p->h_ws);
    hipFree(p->part_ws);
    hipFree(p->obs_ws);
    hipFree(p->done_ws);
    fft_plan_free(p);
    prof_drain(p, p->prof_pending.size());
    for (hipEvent_t e : p->prof_free) hipEventDestroy(e);
    delete p;
    return DDMC_OK;
}

ddmc_status ddmc_plan_create(int32_t L, int32_t M, int32_t R_max, ddmc_prec prec, ddmc_field_algo algo,
                             const double *W64, ddmc_plan **out)
{
    if (!out) return fail(DDMC_EINVAL, "ddmc_plan_create: out is NULL");
    *out = nullptr;
    if (L < 2 || L > 4096) return fail(DDMC_EINVAL, "ddmc_plan_create: L must be in [2, 4096]");
    if (M < -1 || M > 1024) return fail(DDMC_EINVAL, "ddmc_plan_create: M must be -1 (all images) or in [0, 1024]");
    if (R_max < 1 || R_max > 65535) return fail(DDMC_EINVAL, "ddmc_plan_create: R_max must be in [1, 65535]");
    if (prec != DDMC_F64 && prec != DDMC_F32) return fail(DDMC_EINVAL, "ddmc_plan_create: unknown precision");
    if (algo != DDMC_FIELD_AUTO && algo != DDMC_FIELD_DIRECT && algo != DDMC_FIELD_FFT && algo != DDMC_FIELD_FFT_LDS)
        return fail(DDMC_EINVAL, "ddmc_plan_create: unknown field algorithm");
    if (!W64) return fail(DDMC_EINVAL, "ddmc_plan_create: W64 is NULL");
    const bool sweep_lds = algo == DDMC_FIELD_FFT_LDS;
    if (sweep_lds && !(fft_supported(L, prec) && lds_sweep_ok(L, prec)))
        return fail(DDMC_EUNSUPPORTED, "ddmc_plan_create: sweeps in one workgroup need L in {8, 16, 24, 32, 48, 64} "
                                       "(FP64: up to 48)");
    if (sweep_lds) algo = DDMC_FIELD_FFT;
    if (algo == DDMC_FIELD_FFT && !fft_supported(L, prec))
        return fail(DDMC_EUNSUPPORTED, "ddmc_plan_create: the FFT field needs L = 2^a in [8, 512] or 3 * 2^a in "
                                       "[24, 384] (FP64: up to 384)");
    if (algo == DDMC_FIELD_AUTO) algo = fft_supported(L, prec) ? DDMC_FIELD_FFT : DDMC_FIELD_DIRECT;

    ddmc_plan *p = new (std::nothrow) ddmc_plan();
    if (!p) return fail(DDMC_ENOMEM, "ddmc_plan_create: host allocation failed");
    p->L = L;
    p->M = M;
    p->R_max = R_max;
    p->prec = prec;
    p->algo = algo;
    p->sweep_lds = sweep_lds;
    hipGetDevice(&p->device);
    const size_t N = (size_t)L * L;
    const size_t es = elem_size(prec);
    const plan_sizes z = plan_sizes_of(L, R_max, prec, algo);
    ddmc_status st = DDMC_OK;
    auto alloc = [&](void **ptr, size_t bytes, const char *what) {
        if (st != DDMC_OK || bytes == 0) return;
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            *ptr = nullptr;
            st = fail(DDMC_ENOMEM, std::string("ddmc_plan_create: cannot allocate ") + what);
        }
    };
    alloc(&p->W, z.W, "kernel copy");
    alloc(&p->h_ws, z.h, "field workspace");
    alloc(&p->obs_ws, z.obs, "observables workspace");
    alloc((void **)&p->done_ws, z.done, "completion counters");
    if (st == DDMC_OK) {
        hipError_t e = hipMemset(p->done_ws, 0, z.done);
        if (e != hipSuccess) st = hip_check(e, "ddmc_plan_create: workspace clear");
    }
    if (algo == DDMC_FIELD_DIRECT) {
        p->part_elems = z.part / es;
        alloc(&p->part_ws, z.part, "direct-sum partials");
    }
    if (st == DDMC_OK) {
        hipError_t e = prec == DDMC_F64
                           ? launch_convert_kernel<double>(L, W64, reinterpret_cast<double *>(p->W), nullptr)
                           : launch_convert_kernel<float>(L, W64, reinterpret_cast<float *>(p->W), nullptr);
        if (e == hipSuccess) {
            for (int c = 0; c < 4 && e == hipSuccess; ++c)
                e = hipMemcpy(&p->W0[c], W64 + (size_t)c * N, sizeof(double), hipMemcpyDeviceToHost);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) st = hip_check(e, "ddmc_plan_create");
    }
    if (st == DDMC_OK && algo == DDMC_FIELD_FFT)
        st = prec == DDMC_F64 ? fft_plan_init<double>(p, W64) : fft_plan_init<float>(p, W64);
    if (st != DDMC_OK) {
        ddmc_plan_destroy(p);
        return st;
    }
    *out = p;
    return DDMC_OK;
}

ddmc_status ddmc_plan_device_bytes(int32_t L, int32_t R_max, ddmc_prec prec, ddmc_field_algo algo, uint64_t *bytes)
{
    if (!bytes) return fail(DDMC_EINVAL, "ddmc_plan_device_bytes: bytes is NULL");
    if (L < 2 || L > 4096 || R_max < 1 || R_max > 65535)
        return fail(DDMC_EINVAL, "ddmc_plan_device_bytes: L must be in [2, 4096] and R_max in [1, 65535]");
    if (prec != DDMC_F64 && prec != DDMC_F32) return fail(DDMC_EINVAL, "ddmc_plan_device_bytes: unknown precision");
    if (algo != DDMC_FIELD_AUTO && algo != DDMC_FIELD_DIRECT && algo != DDMC_FIELD_FFT && algo != DDMC_FIELD_FFT_LDS)
        return fail(DDMC_EINVAL, "ddmc_plan_device_bytes: unknown field algorithm");
    if (algo == DDMC_FIELD_FFT_LDS) {
        if (!(fft_supported(L, prec) && lds_sweep_ok(L, prec)))
            return fail(DDMC_EUNSUPPORTED, "ddmc_plan_device_bytes: sweeps in one workgroup do not support this L");
        algo = DDMC_FIELD_FFT;
    }
    if (algo == DDMC_FIELD_FFT && !fft_supported(L, prec))
        return fail(DDMC_EUNSUPPORTED, "ddmc_plan_device_bytes: the FFT field does not support this L");
    if (algo == DDMC_FIELD_AUTO) algo = fft_supported(L, prec) ? DDMC_FIELD_FFT : DDMC_FIELD_DIRECT;
    size_t b = plan_sizes_of(L, R_max, prec, algo).total();
    if (algo == DDMC_FIELD_FFT) b += fft_plan_bytes(L, R_max, prec);
    *bytes = (uint64_t)b;
    return DDMC_OK;
}

ddmc_status ddmc_plan_algo(const ddmc_plan *p, ddmc_field_algo *algo)
{
    if (!valid_plan(p) || !algo) return fail(DDMC_EINVAL, "ddmc_plan_algo: NULL argument");
    *algo = p->sweep_lds ? DDMC_FIELD_FFT_LDS : p->algo;
    return DDMC_OK;
}

ddmc_status ddmc_plan_profile(ddmc_plan *p, int32_t enable)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "ddmc_plan_profile: invalid plan");
    prof_drain(p, p->prof_pending.size());
    for (int k = 0; k < DDMC_KERNEL_COUNT; ++k) {
        p->prof_ms[k] = 0.0;
        p->prof_n[k] = 0;
    }
    p->prof = enable != 0;
    return DDMC_OK;
}

ddmc_status ddmc_plan_profile_read(ddmc_plan *p, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!valid_plan(p) || !total_ms || !launches) return fail(DDMC_EINVAL, "ddmc_plan_profile_read: NULL argument");
    if (kernel < 0 || kernel >= DDMC_KERNEL_COUNT) return fail(DDMC_EINVAL, "ddmc_plan_profile_read: bad kernel id");
    prof_drain(p, p->prof_pending.size());
    *total_ms = p->prof_ms[kernel];
    *launches = p->prof_n[kernel];
    return DDMC_OK;
}

ddmc_status replica_params_upload(int32_t R, const ddmc_replica_params *host, ddmc_replica_params *dev,
                                  void *stream)
{
    if (R < 0) return fail(DDMC_EINVAL, "replica_params_upload: R must be >= 0");
    if (R == 0) return DDMC_OK;
    if (!host || !dev) return fail(DDMC_EINVAL, "replica_params_upload: NULL pointer");
    for (int r = 0; r < R; ++r) {
        const ddmc_replica_params &q = host[r];
        const bool T_ok = q.T > 0.0 && !isnan(q.T);
        const bool fin = isfinite(q.J) && isfinite(q.K2) && isfinite(q.K4) && isfinite(q.g);
        if (!T_ok || !fin || (q.model != DDMC_HEISENBERG && q.model != DDMC_ISING))
            return fail(DDMC_EINVAL, "replica_params_upload: replica " + std::to_string(r) +
                                         " has T <= 0, a non-finite parameter or an unknown model");
    }
    return hip_check(launch_params_store(R, host, dev, (hipStream_t)stream), "replica_params_upload");
}

ddmc_status local_field(ddmc_plan *p, int32_t R, const void *s, void *h, int32_t color, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "local_field: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (color < -1 || color > 1) return fail(DDMC_EINVAL, "local_field: color must be -1, 0 or 1");
    if (color >= 0 && (p->L & 1)) return fail(DDMC_EINVAL, "local_field: a colour needs L even");
    if (R == 0) return DDMC_OK;
    if (!s || !h) return fail(DDMC_EINVAL, "local_field: NULL spin or field pointer");
    if (s == h) return fail(DDMC_EINVAL, "local_field: s and h must not overlap");
    hipStream_t st = (hipStream_t)stream;
    if (p->prec == DDMC_F64)
        return field_dispatch<double>(p, R, (const double *)s, (double *)h, color, st);
    return field_dispatch<float>(p, R, (const float *)s, (float *)h, color, st);
}

ddmc_status init_spins(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "init_spins: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (R == 0) return DDMC_OK;
    if (!params || !s) return fail(DDMC_EINVAL, "init_spins: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t he = p->prec == DDMC_F64 ? launch_init_spins<double>(p, R, params, (double *)s, st)
                                        : launch_init_spins<float>(p, R, params, (float *)s, st);
    return hip_check(he, "init_spins launch");
}

ddmc_status metropolis_sweep(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s,
                             uint64_t sweep0, int32_t nsweeps, uint64_t *accepted, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "metropolis_sweep: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (p->L & 1) return fail(DDMC_EINVAL, "metropolis_sweep: L must be even for the checkerboard");
    if (nsweeps < 0) return fail(DDMC_EINVAL, "metropolis_sweep: nsweeps must be >= 0");
    if (sweep0 + (uint64_t)nsweeps > 0x100000000ull)
        return fail(DDMC_EINVAL, "metropolis_sweep: sweep indices must stay below 2^32");
    if (R == 0 || nsweeps == 0) return DDMC_OK;
    if (!params || !s) return fail(DDMC_EINVAL, "metropolis_sweep: NULL pointer");
    return sweep_dispatch(p, R, params, s, nullptr, sweep0, nsweeps, accepted, nullptr, nullptr,
                          (hipStream_t)stream);
}

ddmc_status metropolis_sweep_dev(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s,
                                 uint64_t *sweep_counter, int32_t nsweeps, uint64_t *accepted, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "metropolis_sweep_dev: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (p->L & 1) return fail(DDMC_EINVAL, "metropolis_sweep_dev: L must be even for the checkerboard");
    if (nsweeps < 0) return fail(DDMC_EINVAL, "metropolis_sweep_dev: nsweeps must be >= 0");
    if (!sweep_counter) return fail(DDMC_EINVAL, "metropolis_sweep_dev: NULL sweep counter");
    if (R == 0 || nsweeps == 0) return DDMC_OK;
    if (!params || !s) return fail(DDMC_EINVAL, "metropolis_sweep_dev: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    return sweep_dispatch(p, R, params, s, sweep_counter, 0, nsweeps, accepted, nullptr, nullptr, st);
}

ddmc_status metropolis_sweep_multi(int32_t ngroups, ddmc_plan *const *plans, const int32_t *R,
                                   const ddmc_replica_params *const *params, void *const *s,
                                   uint64_t *const *sweep_counter, int32_t nsweeps, uint64_t *const *accepted,
                                   void *stream)
{
    if (ngroups < 1 || ngroups > DDMC_MULTI_MAX_GROUPS)
        return fail(DDMC_EINVAL, "metropolis_sweep_multi: ngroups must be in [1, DDMC_MULTI_MAX_GROUPS]");
    if (!plans || !R || !params || !s || !sweep_counter)
        return fail(DDMC_EINVAL, "metropolis_sweep_multi: NULL argument array");
    if (nsweeps < 0) return fail(DDMC_EINVAL, "metropolis_sweep_multi: nsweeps must be >= 0");
    ddmc_plan *gp[DDMC_MULTI_MAX_GROUPS];
    int gR[DDMC_MULTI_MAX_GROUPS];
    const ddmc_replica_params *gprm[DDMC_MULTI_MAX_GROUPS];
    void *gs[DDMC_MULTI_MAX_GROUPS];
    uint64_t *gctr[DDMC_MULTI_MAX_GROUPS], *gacc[DDMC_MULTI_MAX_GROUPS];
    int n = 0;
    ddmc_prec prec = DDMC_F32;
    for (int k = 0; k < ngroups; ++k) {
        ddmc_plan *p = plans[k];
        if (!valid_plan(p) || !p->sweep_lds)
            return fail(DDMC_EINVAL, "metropolis_sweep_multi: every plan must be a DDMC_FIELD_FFT_LDS plan");
        if (k > 0 && p->prec != plans[0]->prec)
            return fail(DDMC_EINVAL, "metropolis_sweep_multi: the plans must share one precision");
        prec = p->prec;
        ddmc_status e = check_R(p, R[k]);
        if (e != DDMC_OK) return e;
        if (R[k] == 0) continue;
        if (!params[k] || !s[k] || !sweep_counter[k])
            return fail(DDMC_EINVAL, "metropolis_sweep_multi: NULL pointer of group " + std::to_string(k));
        gp[n] = p;
        gR[n] = R[k];
        gprm[n] = params[k];
        gs[n] = s[k];
        gctr[n] = sweep_counter[k];
        gacc[n] = accepted ? accepted[k] : nullptr;
        ++n;
    }
    if (n == 0 || nsweeps == 0) return DDMC_OK;
    hipStream_t st = (hipStream_t)stream;
    if (prec == DDMC_F64) {
        double *ss[DDMC_MULTI_MAX_GROUPS];
        for (int k = 0; k < n; ++k) ss[k] = (double *)gs[k];
        return lds_sweep<double>(n, gp, gR, gprm, ss, gctr, 0, nsweeps, gacc, nullptr, nullptr, st);
    }
    float *ss[DDMC_MULTI_MAX_GROUPS];
    for (int k = 0; k < n; ++k) ss[k] = (float *)gs[k];
    return lds_sweep<float>(n, gp, gR, gprm, ss, gctr, 0, nsweeps, gacc, nullptr, nullptr, st);
}

ddmc_status metropolis_sample(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s,
                              uint64_t *sweep_counter, int32_t nsweeps, double *obs, double *eta_acc,
                              uint64_t *accepted, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "metropolis_sample: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (p->L & 1) return fail(DDMC_EINVAL, "metropolis_sample: L must be even for the checkerboard");
    if (nsweeps < 0) return fail(DDMC_EINVAL, "metropolis_sample: nsweeps must be >= 0");
    if (!sweep_counter) return fail(DDMC_EINVAL, "metropolis_sample: NULL sweep counter");
    if (!obs) return fail(DDMC_EINVAL, "metropolis_sample: NULL observables output");
    if (R == 0 || nsweeps == 0) return DDMC_OK;
    if (!params || !s) return fail(DDMC_EINVAL, "metropolis_sample: NULL pointer");
    return sweep_dispatch(p, R, params, s, sweep_counter, 0, nsweeps, accepted, obs, eta_acc, (hipStream_t)stream);
}

ddmc_status metropolis_sweep_coset(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s, int32_t l,
                                   uint64_t *sweep_counter, int32_t nsweeps, uint64_t *accepted, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "metropolis_sweep_coset: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (l < 2 || l > p->L || p->L % l != 0)
        return fail(DDMC_EINVAL, "metropolis_sweep_coset: l must be in [2, L] and divide L");
    if (nsweeps < 0) return fail(DDMC_EINVAL, "metropolis_sweep_coset: nsweeps must be >= 0");
    if (!sweep_counter) return fail(DDMC_EINVAL, "metropolis_sweep_coset: NULL sweep counter");
    if (R == 0 || nsweeps == 0) return DDMC_OK;
    if (!params || !s) return fail(DDMC_EINVAL, "metropolis_sweep_coset: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    if (coset_local_ok(p->L, l, p->prec)) {
        if (p->prec == DDMC_F64)
            return coset_local_sweep<double>(p, R, params, (double *)s, l, sweep_counter, nsweeps, accepted, st);
        return coset_local_sweep<float>(p, R, params, (float *)s, l, sweep_counter, nsweeps, accepted, st);
    }
    if (p->algo == DDMC_FIELD_FFT) {
        if (p->prec == DDMC_F64)
            return fft_sweep_coset<double>(p, R, params, (double *)s, l, sweep_counter, nsweeps, accepted, st);
        return fft_sweep_coset<float>(p, R, params, (float *)s, l, sweep_counter, nsweeps, accepted, st);
    }
    if (p->prec == DDMC_F64)
        return sweep_direct_coset<double>(p, R, params, (double *)s, l, sweep_counter, nsweeps, accepted, st);
    return sweep_direct_coset<float>(p, R, params, (float *)s, l, sweep_counter, nsweeps, accepted, st);
}

ddmc_status parallel_tempering_swap(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, void *s,
                                    const double *obs, const uint64_t *sweep_counter, int32_t parity,
                                    uint64_t *swaps, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "parallel_tempering_swap: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (parity != 0 && parity != 1) return fail(DDMC_EINVAL, "parallel_tempering_swap: parity must be 0 or 1");
    if (R < 2) return DDMC_OK;
    if (!params || !s || !obs || !sweep_counter) return fail(DDMC_EINVAL, "parallel_tempering_swap: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t he = p->prec == DDMC_F64
                        ? launch_pt_swap<double>(p, R, params, (double *)s, obs, sweep_counter, parity, swaps, st)
                        : launch_pt_swap<float>(p, R, params, (float *)s, obs, sweep_counter, parity, swaps, st);
    return hip_check(he, "parallel_tempering_swap launch");
}

ddmc_status coset_error_bound(int32_t L, int32_t l, int32_t all_images, double *eps)
{
    if (!eps) return fail(DDMC_EINVAL, "coset_error_bound: eps is NULL");
    if (L < 2 || L > 4096 || l < 2 || l > L || L % l != 0)
        return fail(DDMC_EINVAL, "coset_error_bound: need 2 <= l <= L <= 4096 with l dividing L");
    if (all_images) {
        // every partner of l Z^2 minus the origin: 2 S / l^3, with S the lattice
        // sum of |r|^-3 over Z^2 minus the origin, 4 zeta(3/2) beta(3/2)
        const double S = 9.0336216831009475;
        *eps = 2.0 * S / ((double)l * l * l);
        return DDMC_OK;
    }
    // the other sites of the coset, each at its nearest image
    const int n = L / l;
    double acc = 0.0;
    for (int b = 0; b < n; ++b) {
        long dy = (long)b * l;
        if (2 * dy > L) dy -= L;
        for (int a = 0; a < n; ++a) {
            long dx = (long)a * l;
            if (2 * dx > L) dx -= L;
            if (dx == 0 && dy == 0) continue;
            const double r = sqrt((double)(dx * dx + dy * dy));
            acc += 2.0 / (r * r * r);
        }
    }
    *eps = acc;
    return DDMC_OK;
}

ddmc_status trial_energies(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, const void *s,
                           const void *h, uint32_t sweep, int32_t color, void *dE, void *u, void *S,
                           void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "trial_energies: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (p->L & 1) return fail(DDMC_EINVAL, "trial_energies: L must be even");
    if (color != 0 && color != 1) return fail(DDMC_EINVAL, "trial_energies: color must be 0 or 1");
    if (R == 0) return DDMC_OK;
    if (!params || !s || !h || !dE || !u) return fail(DDMC_EINVAL, "trial_energies: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t he =
        p->prec == DDMC_F64
            ? launch_trial<double>(p, R, params, (const double *)s, (const double *)h, color, sweep, (double *)dE,
                                   (double *)u, (double *)S, st)
            : launch_trial<float>(p, R, params, (const float *)s, (const float *)h, color, sweep, (float *)dE,
                                  (float *)u, (float *)S, st);
    return hip_check(he, "trial_energies launch");
}

ddmc_status spins_convert(int32_t R, int32_t L, const void *src, ddmc_prec src_prec, void *dst, ddmc_prec dst_prec,
                          void *stream)
{
    if (R < 0 || L < 1 || L > 4096) return fail(DDMC_EINVAL, "spins_convert: bad R or L");
    if ((src_prec != DDMC_F64 && src_prec != DDMC_F32) || (dst_prec != DDMC_F64 && dst_prec != DDMC_F32))
        return fail(DDMC_EINVAL, "spins_convert: unknown precision");
    if (R == 0) return DDMC_OK;
    if (!src || !dst) return fail(DDMC_EINVAL, "spins_convert: NULL pointer");
    const long n = (long)R * 3 * L * L;
    const char *s0 = (const char *)src, *d0 = (const char *)dst;
    const long sb = n * (src_prec == DDMC_F64 ? 8 : 4), db = n * (dst_prec == DDMC_F64 ? 8 : 4);
    if (s0 < d0 + db && d0 < s0 + sb) return fail(DDMC_EINVAL, "spins_convert: src and dst overlap");
    return hip_check(launch_spins_convert(n, src, src_prec == DDMC_F64, dst, dst_prec == DDMC_F64, (hipStream_t)stream),
                     "spins_convert launch");
}

ddmc_status observables(ddmc_plan *p, int32_t R, const ddmc_replica_params *params, const void *s, const void *h,
                        double *out, double *eta_acc, void *stream)
{
    if (!valid_plan(p)) return fail(DDMC_EINVAL, "observables: invalid plan");
    ddmc_status e = check_R(p, R);
    if (e != DDMC_OK) return e;
    if (R == 0) return DDMC_OK;
    if (!params || !s || !out) return fail(DDMC_EINVAL, "observables: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t he = p->prec == DDMC_F64
                        ? launch_observables<double>(p, R, params, (const double *)s, (const double *)h, out,
                                                     eta_acc, st)
                        : launch_observables<float>(p, R, params, (const float *)s, (const float *)h, out,
                                                    eta_acc, st);
    return hip_check(he, "observables launch");
}

ddmc_status observables_noalloc(int32_t L, ddmc_prec prec, int32_t R, const ddmc_replica_params *params,
                                const void *s, const void *h, double *out, double *eta_acc, void *stream)
{
    if (L < 1 || L > 4096) return fail(DDMC_EINVAL, "observables_noalloc: L must be in [1, 4096]");
    if (prec != DDMC_F64 && prec != DDMC_F32) return fail(DDMC_EINVAL, "observables_noalloc: unknown precision");
    if (R < 0 || R > DDMC_NOALLOC_R_MAX)
        return fail(DDMC_EINVAL, "observables_noalloc: R must be in [0, " + std::to_string(DDMC_NOALLOC_R_MAX) +
                                     "] (the static scratch holds that many replicas)");
    if (R == 0) return DDMC_OK;
    if (!params || !s || !out) return fail(DDMC_EINVAL, "observables_noalloc: NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t he = prec == DDMC_F64
                        ? launch_observables_noalloc<double>(L, R, params, (const double *)s, (const double *)h, out,
                                                             eta_acc, st)
                        : launch_observables_noalloc<float>(L, R, params, (const float *)s, (const float *)h, out,
                                                            eta_acc, st);
    return hip_check(he, "observables_noalloc launch");
}

}  // extern "C"
