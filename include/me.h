/*
 * me.h -- C ABI of the MI355X matrix-element library (libme.so).
 *
 * The library evaluates, for every phase-space point of a batch, the squared
 * tree-level matrix element |M|^2 of one fixed partonic process: helicity
 * amplitudes from external and internal wavefunctions for every Feynman
 * diagram, accumulated into colour-flow amplitudes J, the colour sum
 * J^dag C J with the process's constant colour matrix, summed over
 * helicities.  This is the matrix-element step of the paper's event
 * generator (Sec. 2: random numbers -> momenta -> matrix element, with a
 * data-parallel, reentrant, stateless multi-event interface; Sec. 3: the
 * Feynman-diagram code and the colour-matrix quadratic form).
 *
 * Conventions shared by every call:
 *   - Status codes only (ME_OK or a negative ME_E* value); nothing throws,
 *     aborts or exits across the ABI.  me_last_error() gives a thread-local
 *     detail string for the last failure on the calling thread.
 *   - "device pointer" means memory on the current HIP device (e.g. a torch
 *     tensor's data_ptr()); the caller owns every data buffer.  The context
 *     owns its constants and scratch and releases them in me_free().
 *   - Calls that take a stream are asynchronous on that stream (NULL = the
 *     default stream); results are valid once the stream has synchronised.
 *   - Momenta are float64, laid out [nevt][npart][4] with components
 *     (E, px, py, pz) in GeV, particle order as listed for each process.
 *     Inputs are not validated kinematically; NaN/Inf propagate to NaN
 *     outputs without trapping.
 *   - A context is used by one host thread at a time; me_init is thread-safe.
 */
#ifndef ME_H
#define ME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct me_ctx me_ctx;

enum {
    ME_OK = 0,
    ME_EINVAL = -1,   /* null pointer, negative size, wrong argument count */
    ME_EPROCESS = -2, /* unknown process name */
    ME_EDEVICE = -3,  /* HIP runtime failure (detail in me_last_error) */
    ME_ENOMEM = -4,   /* device allocation failed */
    ME_ESTATE = -5    /* call not valid in the context's current state */
};

enum { ME_FP64 = 0, ME_MIXED = 1 };
enum { ME_COLOUR_VALU = 0, ME_COLOUR_MFMA = 1 };

/*
 * me_init -- create a context for one process on the current HIP device.
 * (Paper Sec. 2: the matrix-element library is initialised once per process
 * with the model's couplings and masses, then called on batches of events.)
 *
 * process: "ee_mumu"  e+(1) e-(2) -> mu+(3) mu-(4), s-channel photon + Z
 *          "gg_tt"    g(1) g(2) -> t(3) tbar(4)
 *          "gg_ttg"   g g -> t tbar g(5)
 *          "gg_ttgg"  g g -> t tbar g(5) g(6)
 *          "gg_ttggg" g g -> t tbar g(5) g(6) g(7)
 * couplings: host array {alpha_s, 1/alpha, G_F}, n_couplings == 3
 *            (e.g. {0.118, 132.507, 1.16639e-5}); M_W and sin^2(theta_W)
 *            follow from (alpha, G_F, M_Z).
 * masses:    host array {M_Z, W_Z, M_top, W_top} in GeV, n_masses == 4
 *            (e.g. {91.188, 2.4414, 173.0, 1.4915}); the top width sits on
 *            every internal top line.
 * out_ctx:   receives the new context.
 *
 * Runs the helicity filter once: every helicity combination is evaluated in
 * float64 on a few fixed probe points and those whose contribution is exactly
 * zero on all of them are dropped from later evaluations.  Synchronises the
 * device.  Errors: ME_EINVAL, ME_EPROCESS, ME_EDEVICE, ME_ENOMEM.
 */
int me_init(const char *process, const double *couplings, int n_couplings, const double *masses, int n_masses,
            me_ctx **out_ctx);

/*
 * me_eval -- |M|^2 for nevt points.
 * (Paper Sec. 2: the data-parallel, reentrant, stateless multi-event call of
 * the matrix-element step; Sec. 3: its cost is the Feynman-diagram code plus
 * the colour-matrix quadratic form.)
 * momenta: device pointer, float64 [nevt][npart][4].
 * out_me2: device pointer, float64 [nevt]; receives |M|^2 summed over final
 *          and averaged over initial helicities and colours, divided by the
 *          number of permutations of identical final-state gluons.
 * stream:  hipStream_t (NULL = default stream); no host synchronisation.
 * nevt == 0 launches nothing.  Errors: ME_EINVAL (null pointer, nevt < 0),
 * ME_EDEVICE (launch failure).
 * Reproducibility: results are deterministic for every process except
 * "gg_ttggg", whose kernel adds the contributions of four waves into shared
 * colour-flow amplitudes with atomic float64 adds; its results agree from run
 * to run to rounding (relative 1e-15 level), not bit for bit.
 */
int me_eval(me_ctx *ctx, const double *momenta, int64_t nevt, double *out_me2, void *stream);

/*
 * me_set_precision -- choose the evaluation form of later me_eval calls.
 * (Paper Sec. 3 compares double, float and mixed builds; the mixed form here
 * is float32 amplitudes with a float16 matrix-core colour sum and a float64
 * rerun of events whose estimated error exceeds the tolerance.)
 * ME_FP64 (default): float64 throughout.
 * ME_MIXED: float32 wavefunctions and amplitudes (momentum algebra and
 *   propagator denominators in float64), colour sum as a float16 hi/lo GEMM on
 *   the matrix cores with float32 accumulation, and a calibrated
 *   a-posteriori estimate of each event's relative rounding error (not a
 *   rigorous bound; see me_eval_mixed_diag); every event whose estimate
 *   exceeds rel_tol is recomputed in float64 on the same stream, so each
 *   returned value is expected within rel_tol of the exact float64 result
 *   (measured: all of 2^16 g g -> t tbar g g and 2^12 g g -> t tbar g g g
 *   events at rel_tol = 1e-5).  Processes
 *   without a mixed form (e+e- -> mu+mu-) keep evaluating in float64.
 *   Mixed evaluation keeps a flagged-event index list in the context; it grows
 *   on the first call with a larger nevt (that call synchronises the device).
 * Errors: ME_EINVAL (unknown mode, rel_tol <= 0 for ME_MIXED).
 */
int me_set_precision(me_ctx *ctx, int mode, double rel_tol);

/*
 * me_set_helicity_lanes -- helicity-level parallelism of later float64
 * me_eval calls (the paper's Sec. 2: besides one event per thread, the
 * helicities of one event can be spread over threads, so that fewer events in
 * flight fill the GPU).  lanes: 1 (one lane sums all helicities of its
 * event), 2, 4, 8, 16, 32 or 64 lanes per event; each lane sums every
 * lanes-th filtered helicity and the lanes' partial sums are added when the
 * event is done.  lanes = 0 (the default): chosen per call, the smallest
 * power of two with nevt * lanes >= 65536, at most 64 and at most the number
 * of helicities kept (one lane per event from 65536 events up), and at least
 * a measured per-process floor (8 for "gg_ttgg", 1 otherwise).  The result
 * equals the one-lane result up to the order of the helicity sum.  Applies to
 * the float64 form of me_eval only (the mixed form, its float64 rerun,
 * me_eval_helicities and unweighting keep one lane per event).  Errors:
 * ME_EINVAL (null context, lanes neither 0 nor a power of two up to 64).
 */
int me_set_helicity_lanes(me_ctx *ctx, int lanes);

/*
 * me_set_colour_form -- where later float64 me_eval and me_eval_helicities
 * calls evaluate the colour sum J^dag C J (the colour-matrix quadratic form of
 * the paper's Sec. 3).  ME_COLOUR_VALU (default): per event on the vector
 * ALU, using the symmetry of C.  ME_COLOUR_MFMA: batched over the events of a
 * tile as a float64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64) over
 * block pairs of the symmetric C, from J staged in LDS.  Both give the same
 * result up to rounding; which one is faster depends on the process (the
 * measured choice is the default).  Errors: ME_EINVAL (unknown form),
 * ME_ESTATE (the process has no matrix-core colour form: only "gg_ttgg" and
 * "gg_ttggg" have one).
 */
int me_set_colour_form(me_ctx *ctx, int form);

/*
 * me_eval_mixed_diag -- the mixed form without the float64 rerun, for checks
 * (the precision study of the paper's Sec. 3, per event).
 * out_me2:  device float64 [nevt], the float32-form result of every event.
 * out_err:  device float32 [nevt], the estimated relative error: a calibrated
 *           estimate from the magnitudes of the amplitudes added into each
 *           colour flow, not a rigorous bound (measured against the float64
 *           oracle it is above the actual error of all but about 3 in 10^5
 *           g g -> t tbar g g events, by a factor of 25 at the median).
 * out_flag: device uint8 [nevt], 1 where out_err exceeds the context's
 *           tolerance (the events me_eval would recompute in float64).
 * Errors: ME_EINVAL, ME_ESTATE (process without a mixed form), ME_EDEVICE.
 */
int me_eval_mixed_diag(me_ctx *ctx, const double *momenta, int64_t nevt, double *out_me2, float *out_err,
                       uint8_t *out_flag, void *stream);

/*
 * me_fallback_count -- number of events the last mixed me_eval recomputed in
 * float64.  Synchronises the device (all streams) before it reads the count.
 * 0 before any mixed evaluation.
 */
int me_fallback_count(me_ctx *ctx, int64_t *count);

/* Largest nevt me_eval_mixed_noalloc accepts. */
#define ME_NOALLOC_MAX_NEVT (1 << 20)

/*
 * me_eval_mixed_noalloc -- me_eval in the mixed form (tolerance as set by
 * me_set_precision, default 1e-5; the context's mode is not consulted) with no
 * device allocation: for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * momenta, out_me2, stream: as in me_eval.  The flagged-event counter and
 * index list of the float64 rerun live in a fixed library-owned scratch array
 * on each device (4 MiB + 256 B, allocated at load time, held until the
 * process ends), whose address is looked up when a context is created on
 * that device.  Every call on one GPU shares that array and the last call's
 * contents remain; the counter is cleared by a kernel at the start of each
 * call, so two calls that overlap on one GPU (different streams, or threads)
 * race and must be ordered by the caller.  Processes without a mixed form
 * (e+e- -> mu+mu-) are evaluated in float64 and touch no scratch.
 * me_fallback_count does not report the events of this call.
 * Errors: ME_EINVAL (null pointer, nevt < 0, nevt > ME_NOALLOC_MAX_NEVT),
 * ME_ESTATE (current device is not the context's), ME_EDEVICE.
 */
int me_eval_mixed_noalloc(me_ctx *ctx, const double *momenta, int64_t nevt, double *out_me2, void *stream);

/*
 * me_eval_helicities -- per-helicity contributions, for checks (the helicity
 * sum of the paper's Sec. 2 taken apart).
 * out_qhel: device pointer, float64 [nevt][nhel]; entry h receives
 *           J_h^dag C J_h (before averaging) for every helicity combination
 *           h in 0..nhel-1 (particle i has helicity + when bit (npart-1-i)
 *           of h is set), including those the filter dropped.
 * out_me2:  as in me_eval, but summed over all helicities (no filter).
 */
int me_eval_helicities(me_ctx *ctx, const double *momenta, int64_t nevt, double *out_me2, double *out_qhel,
                       void *stream);

/*
 * me_info -- static properties of the context's process (diagrams, colour
 * flows, helicities: the sizes behind the paper's Sec. 3 cost discussion).
 * Any output pointer may be NULL.  flops_per_event: the algorithmic
 * floating-point operation count of one event over the good helicities
 * (diagram program + colour sum; FMA counted as two operations).
 */
int me_info(const me_ctx *ctx, int *npart, int *ndiag, int *ncol, int *nhel, int *nhel_good,
            double *flops_per_event);

/*
 * Multi-channel weights (the paper's Sec. 2: the multi-channel integration of
 * the event generator processes events of different channels in one
 * matrix-element kernel; a channel is a Feynman diagram, and the event's
 * weight in its channel is that diagram's share of the sum over diagrams of
 * |A_d|^2, the single-diagram enhancement).
 *
 * me_channels -- *nchan receives the number of channels of the context's
 *   process: its Feynman diagrams whose gluons meet at three-point vertices
 *   only (diagrams with a four-gluon vertex are not channels); 0 when the
 *   process has no multi-channel form ("gg_tt", "gg_ttg", "gg_ttgg" have one).
 * me_channel_desc -- the descriptor of channel `chan` into buf (NUL-terminated,
 *   buflen bytes): the gluon trees of the diagram in order along the top line
 *   from ubar(p3) to v(p4), separated by '|', each tree written as nested
 *   "(x,y)" with the subtree holding the smaller gluon label first; gluon
 *   labels 0, 1 are the incoming gluons, 2, 3, ... the final ones in particle
 *   order.  Channels are numbered in the lexicographic order of descriptors.
 *   Errors: ME_EINVAL (chan out of range, buffer too short), ME_ESTATE.
 * me_eval_multichannel -- for nevt points and a channel per point:
 *   momenta: device float64 [nevt][npart][4]; chan: device int32 [nevt];
 *   out_me2: device float64 [nevt], |M|^2 as from me_eval;
 *   out_alpha: device float64 [nevt], sum over helicities of |A_chan|^2
 *   divided by the same sum over all channel diagrams (colour factors
 *   stripped so that every colour-flow coefficient has unit modulus); 0 when
 *   chan is outside 0 .. nchan - 1.  The evaluation is float64 with one
 *   amplitude per Feynman diagram (no merged currents).  Errors: ME_EINVAL,
 *   ME_ESTATE (no multi-channel form), ME_EDEVICE.
 */
int me_channels(const me_ctx *ctx, int *nchan);
int me_channel_desc(const me_ctx *ctx, int chan, char *buf, int buflen);
int me_eval_multichannel(me_ctx *ctx, const double *momenta, const int32_t *chan, int64_t nevt, double *out_me2,
                         double *out_alpha, void *stream);

/*
 * me_flops -- the floating-point operation counts behind me_info's total, per
 * helicity (any output may be NULL): amp_per_hel, the diagram part (external
 * wavefunctions, currents, amplitudes, accumulation into J) with every
 * wavefunction computed once; colour_per_hel, the colour sum J^dag N J in the
 * symmetric form the float64 kernels evaluate; executed_per_hel, the diagram
 * part as the float64 kernel executes it (wavefunctions recomputed under its
 * register budget included, all waves of a workgroup kernel together).  FMA
 * counts as two operations.  These are the algorithmic counts of the
 * roofline accounting (the paper's Sec. 3 splits the cost the same way:
 * Feynman-diagram code and the colour-matrix quadratic form).
 */
int me_flops(const me_ctx *ctx, double *amp_per_hel, double *colour_per_hel, double *executed_per_hel);

/* me_good_helicities -- copy the filtered helicity indices (host array of at
 * least nhel ints); *count receives how many there are.  The filter itself is
 * not in the paper (see me_init). */
int me_good_helicities(const me_ctx *ctx, int *out, int *count);

/* me_free -- release the context (NULL is allowed). Synchronises the device. */
int me_free(me_ctx *ctx);

const char *me_strerror(int status);
const char *me_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ME_H */
