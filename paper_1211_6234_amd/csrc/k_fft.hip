// k_fft.hip -- FFT form of the local dipolar field (placeholder until the
// FFT kernels land: every entry reports the size as unsupported).
#include "internal.hpp"

namespace ddmc {

bool fft_supported(int) { return false; }

template <typename T> ddmc_status fft_plan_init(ddmc_plan *, const double *)
{
    return fail(DDMC_EUNSUPPORTED, "FFT field not available");
}
template <typename T> ddmc_status fft_field(ddmc_plan *, int, const T *, T *, int, hipStream_t)
{
    return fail(DDMC_EUNSUPPORTED, "FFT field not available");
}
template <typename T>
ddmc_status fft_sweep(ddmc_plan *, int, const ddmc_replica_params *, T *, uint64_t, int, uint64_t *, hipStream_t)
{
    return fail(DDMC_EUNSUPPORTED, "FFT field not available");
}
void fft_plan_free(ddmc_plan *) {}

template ddmc_status fft_plan_init<float>(ddmc_plan *, const double *);
template ddmc_status fft_plan_init<double>(ddmc_plan *, const double *);
template ddmc_status fft_field<float>(ddmc_plan *, int, const float *, float *, int, hipStream_t);
template ddmc_status fft_field<double>(ddmc_plan *, int, const double *, double *, int, hipStream_t);
template ddmc_status fft_sweep<float>(ddmc_plan *, int, const ddmc_replica_params *, float *, uint64_t, int,
                                      uint64_t *, hipStream_t);
template ddmc_status fft_sweep<double>(ddmc_plan *, int, const ddmc_replica_params *, double *, uint64_t, int,
                                       uint64_t *, hipStream_t);

}  // namespace ddmc
