// me_unweight.hip -- two-stage unweighting driven by the surrogate network
// (Danziger, Janssen, Schumann, Siegert, SciPost Phys. 12 (2022) 164): the
// network's weight decides a first accept/reject, the exact float64 matrix
// element of the survivors a second one, and the output weights
// max(1, s/s_max) max(1, (w/s)/r_max) keep every point's expected
// contribution proportional to its exact weight w.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/mlp.h"
#include "me_internal.h"

#define HCHK(expr)                                                                                   \
    do {                                                                                             \
        hipError_t _e = (expr);                                                                      \
        if (_e != hipSuccess) return me_fail(ME_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

// Wave-aggregated append of `take` lanes to list[*count]: returns the slot.
__device__ __forceinline__ int append_slot(bool take, int* count) {
    const unsigned long long ballot = __ballot(take);
    if (!ballot) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)ballot) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(ballot));
    base = __shfl(base, leader);
    return take ? base + __popcll(ballot & ((1ull << lane) - 1ull)) : -1;
}

__global__ void k_uw_zero(int* count) {
    if (threadIdx.x < 2 && blockIdx.x == 0) count[threadIdx.x] = 0;
}

// stage 1: s = exp(sigma y + mu) w_ps; survivors appended to idx1 (count[0])
__global__ void k_uw_stage1(const float* __restrict__ y, const double* __restrict__ w_ps,
                            const double* __restrict__ u, int64_t n, double mu, double sigma, double s_max,
                            double* __restrict__ s_out, int* __restrict__ idx1, int* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool take = false;
    if (i < n) {
        const double s = exp(sigma * (double)y[i] + mu) * w_ps[i];
        s_out[i] = s;
        take = u[2 * i] < fmin(1.0, s / s_max);
    }
    const int slot = append_slot(take, &count[0]);
    if (take) idx1[slot] = (int)i;
}

// stage 2 over the survivors: exact weight from the float64 matrix element
__global__ void k_uw_stage2(const int* __restrict__ idx1, const double* __restrict__ me2,
                            const double* __restrict__ w_ps, const double* __restrict__ s_in,
                            const double* __restrict__ u, double s_max, double r_max, int* __restrict__ count,
                            int32_t* __restrict__ out_idx, double* __restrict__ out_w) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    bool take = false;
    int i = 0;
    double wt = 0.0;
    if (j < count[0]) {
        i = idx1[j];
        const double s = s_in[i];
        const double r = me2[i] * w_ps[i] / s;
        take = u[2 * (int64_t)i + 1] < fmin(1.0, r / r_max);
        wt = fmax(1.0, s / s_max) * fmax(1.0, r / r_max);
    }
    const int slot = append_slot(take, &count[1]);
    if (take) {
        out_idx[slot] = i;
        out_w[slot] = wt;
    }
}

static int ensure_uw(me_ctx* c, int64_t n, int n_in) {
    if (n <= c->uw_cap) return ME_OK;
    HCHK(hipDeviceSynchronize());
    void* bufs[] = {c->uw_x, c->uw_y, c->uw_s, c->uw_me2, c->uw_idx1};
    for (void* b : bufs)
        if (b) HCHK(hipFree(b));
    HCHK(hipMalloc(&c->uw_x, n * n_in * sizeof(float)));
    HCHK(hipMalloc(&c->uw_y, n * sizeof(float)));
    HCHK(hipMalloc(&c->uw_s, n * sizeof(double)));
    HCHK(hipMalloc(&c->uw_me2, n * sizeof(double)));
    HCHK(hipMalloc(&c->uw_idx1, n * sizeof(int)));
    c->uw_cap = n;
    return ME_OK;
}

extern "C" int unweight_two_stage(me_ctx* c, me_mlp* mlp, const double* momenta, const double* w_ps, int64_t n,
                                  const double* uniforms, double y_mu, double y_sigma, double s_max, double r_max,
                                  int32_t* out_idx, double* out_w, int32_t* out_count, void* stream) {
    if (!c || !mlp || n < 0) return me_fail(ME_EINVAL, "unweight_two_stage: null argument or negative n");
    if (!(s_max > 0) || !(r_max > 0)) return me_fail(ME_EINVAL, "unweight_two_stage: s_max, r_max must be positive");
    if (!out_count) return me_fail(ME_EINVAL, "unweight_two_stage: null out_count");
    if (n > 0x7fffffffLL) return me_fail(ME_EINVAL, "unweight_two_stage: n above 2^31 - 1");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_uw_zero, dim3(1), dim3(64), 0, s, out_count);
    if (n == 0) {
        HCHK(hipGetLastError());
        return ME_OK;
    }
    if (!momenta || !w_ps || !uniforms || !out_idx || !out_w) return me_fail(ME_EINVAL, "unweight_two_stage: null buffer");
    const int npart = c->proc->npart;
    if (mlp_n_in(mlp) != 4 * npart) return me_fail(ME_EINVAL, "unweight_two_stage: network inputs != 4 npart");
    int rc = ensure_uw(c, n, 4 * npart);
    if (rc != ME_OK) return rc;
    rc = me_features(momenta, n, npart, c->uw_x, s);
    if (rc != ME_OK) return rc;
    rc = mlp_forward_internal(mlp, c->uw_x, n, c->uw_y, s);
    if (rc != ME_OK) return rc;
    const dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_uw_stage1, grid, dim3(256), 0, s, c->uw_y, w_ps, uniforms, n, y_mu, y_sigma, s_max, c->uw_s,
                       c->uw_idx1, out_count);
    // exact float64 matrix element of the stage-1 survivors only
    HCHK(c->proc->launch_f64_idx(momenta, n, c->uw_me2, c->d_good, c->nhel_good, c->prm, c->uw_idx1, out_count, s));
    hipLaunchKernelGGL(k_uw_stage2, grid, dim3(256), 0, s, c->uw_idx1, c->uw_me2, w_ps, c->uw_s, uniforms, s_max,
                       r_max, out_count, out_idx, out_w);
    HCHK(hipGetLastError());
    return ME_OK;
}
