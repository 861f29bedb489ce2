// Persistent, temporally blocked sweep.
#include "rbgs_blocked.h"
#include "rbgs_internal.h"

namespace rbgs {

size_t blocked_state_bytes(int, int) { return 256; }

int validate_blocked_opts(int, int, int, std::string*) { return RBGS_OK; }

int auto_kernel(int, size_t) { return RBGS_KERNEL_PLAIN; }

BlockedParams blocked_params(int, size_t, const rbgs_sweep_opts*) { return BlockedParams{}; }

template <typename T>
hipError_t run_blocked(T*, T*, const T*, const T*, int, int64_t, T, int, const BlockedParams&,
                       void*, size_t, hipStream_t, int*, int*) {
    return hipErrorNotSupported;
}

template hipError_t run_blocked<double>(double*, double*, const double*, const double*, int,
                                        int64_t, double, int, const BlockedParams&, void*, size_t,
                                        hipStream_t, int*, int*);
template hipError_t run_blocked<float>(float*, float*, const float*, const float*, int, int64_t,
                                       float, int, const BlockedParams&, void*, size_t,
                                       hipStream_t, int*, int*);

int blocked_check_error(void*, hipStream_t, std::string*) { return RBGS_OK; }

}  // namespace rbgs
