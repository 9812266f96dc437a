// me_internal.h -- library-internal state shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/me.h"
#include "me_launch.h"

// Devices the allocation-free entry point keeps a scratch address for.
#define ME_MAX_DEVICES 64

// Records the detail string for me_last_error() and returns code.
int me_fail(int code, const std::string& msg);

struct me_ctx {
    const me_process_desc* proc;
    me_params prm;
    int device;
    int nhel_good;
    std::vector<int> good;  // host copy of the filtered helicities
    int* d_good;            // device copy
    int* d_all;             // device list 0..nhel-1
    int mode;               // ME_FP64 or ME_MIXED
    int hel_lg;             // float64 form: 2^hel_lg lanes per event (helicity parallelism), -1 automatic
    int colour_form;        // float64 form: ME_COLOUR_VALU or ME_COLOUR_MFMA
    double tol;             // mixed form: per-event relative error tolerance
    // scratch of the mixed form: flagged-event counter and index list
    int* d_count;
    int* d_idx;
    int64_t idx_cap;
    // scratch of two-stage unweighting
    float* uw_x;
    float* uw_y;
    double* uw_s;
    double* uw_me2;
    int* uw_idx1;
    int64_t uw_cap;
};

struct me_mlp;
int mlp_forward_internal(me_mlp* p, const float* x, int64_t n, float* y, hipStream_t s);
int mlp_n_in(const me_mlp* p);
