// me_launch.h -- host-side process table shared by the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "me_process.h"

#define ME_BLOCK 64

typedef hipError_t (*me_launch_fn)(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                   const me_params& prm, double* qhel, hipStream_t stream);

enum { ME_KIND_EE = 0, ME_KIND_GG = 1 };

struct me_process_desc {
    const char* name;
    int kind;
    int npart, ndiag, ncol, nhel;
    double flops_amp, flops_colour;  // per helicity
    me_launch_fn launch_f64;
};

const me_process_desc* me_find_process(const char* name);
