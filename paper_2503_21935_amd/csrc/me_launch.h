// me_launch.h -- host-side process table shared by the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "me_process.h"

#define ME_BLOCK 64

// lg: 2^lg lanes per event, each summing every 2^lg-th helicity (0 <= lg <= 6).
typedef hipError_t (*me_launch_fn)(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                   const me_params& prm, double* qhel, int lg, hipStream_t stream);

// Indexed variant: evaluate events idx[0..*count) only (count on the device).
typedef hipError_t (*me_launch_idx_fn)(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                       const me_params& prm, const int* idx, const int* count,
                                       hipStream_t stream);

// Mixed-precision form: float32 amplitudes, float16 hi/lo MFMA colour sum,
// per-event error estimate; flagged events appended to flag_idx.
typedef hipError_t (*me_launch_mixed_fn)(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                         const me_params& prm, float tol, float cest, int* flag_count,
                                         int* flag_idx, float* err_out, unsigned char* flag_out,
                                         hipStream_t stream);

// Multi-channel form: |M|^2 and the single-diagram weight of each event's channel.
typedef hipError_t (*me_launch_mc_fn)(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                      const me_params& prm, const int* chan, double* alpha, hipStream_t stream);

enum { ME_KIND_EE = 0, ME_KIND_GG = 1, ME_KIND_QEW = 2 };

struct me_process_desc {
    const char* name;
    int kind;
    int npart, ndiag, ncol, nhel;
    double flops_amp, flops_colour;  // per helicity, algorithmic
    double flops_executed;           // per helicity, as the kernel executes it (recomputation included)
    me_launch_fn launch_f64;
    me_launch_idx_fn launch_f64_idx;
    me_launch_mixed_fn launch_mixed;  // nullptr: the process has no mixed form
    double mixed_cest;                // calibration of the amplitude error estimate
    double colour_err;                // a-priori error of the float16 hi/lo colour sum
    me_launch_fn launch_f64_cm;       // float64 with the colour sum on the matrix cores (nullptr: none)
    me_launch_mc_fn launch_mc;        // multi-channel form (nullptr: none)
    int nchan;                        // its channels
    const char* const* chan_desc;     // their descriptors
};

const me_process_desc* me_find_process(const char* name);
