/*
 * ps.h -- C ABI of the phase-space sampling step in libme.so.
 *
 * The paper's generator makes three data-parallel steps per event: random
 * numbers, momenta from them, the matrix element (Sec. 2, overview of the
 * architecture); its outlook (Sec. 3) names phase-space sampling on the GPU
 * as the next step once the matrix element is fast.  ps_rambo does the first
 * two steps on the GPU for flat phase space, so that points need not be made
 * on the host and copied over.
 *
 * Conventions as in me.h (status codes, caller-owned device buffers,
 * asynchronous on the given stream, me_last_error() for details).
 */
#ifndef PS_H
#define PS_H

#include <stdint.h>

#include "me.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * ps_rambo -- nevt flat phase-space points at fixed partonic sqrt(s).
 *
 * roots:   sqrt(s) in GeV (> sum of the masses).
 * masses:  host array of nfinal final-state masses (GeV, >= 0).
 * nfinal:  number of final-state particles, 2..8.
 * seed, first_event: event e of this call uses the random stream of event
 *          first_event + e: Philox4x32-10 (Salmon et al., SC'11) with key =
 *          seed (low word, high word) and counter (event low word, event high
 *          word, block b, 0); block b gives uniforms 2b and 2b + 1, each made
 *          from 64 bits as ((w0 * 2^32 + w1) >> 11 + 1/2) * 2^-53 in (0, 1).
 *          Particle i takes uniforms 4i .. 4i + 3.  Results therefore do not
 *          depend on how a sample is split into calls.
 * momenta: device float64 [nevt][nfinal + 2][4], 16-byte aligned, (E, px,
 *          py, pz): particles 0 and 1 are the incoming partons
 *          (sqrt(s)/2)(1, 0, 0, +1) and (sqrt(s)/2)(1, 0, 0, -1), then the
 *          final state from the RAMBO map (Kleiss, Stirling, Ellis, Comput.
 *          Phys. Commun. 40 (1986) 359), massive momenta by the rescaling of
 *          the 3-momenta that restores the total energy; every final
 *          energy is sqrt(m^2 + |k|^2).
 * weights: device float64 [nevt] or NULL; the phase-space weight of each
 *          point: the flat massless n-body volume (2 pi)^(4-3n) (pi/2)^(n-1)
 *          s^(n-2) / ((n-1)! (n-2)!), times the RAMBO mass factor.
 * Errors: ME_EINVAL (sizes, masses, alignment), ME_EDEVICE.
 */
int ps_rambo(double roots, const double *masses, int nfinal, uint64_t seed, int64_t first_event, int64_t nevt,
             double *momenta, double *weights, void *stream);

/*
 * ps_multichannel -- nevt phase-space points for a final state with a lepton
 * pair, sampled from three channels and weighted by the multi-channel weight.
 * The paper names faster phase-space sampling on the GPU as the next step
 * (Sec. 3, outlook); for a pair produced through a photon or a Z boson, flat
 * sampling wastes most points away from the pair-mass peaks.
 *
 * Channels (alpha normalised to sum 1):
 *   0: flat RAMBO over the nfinal particles (as ps_rambo, massless);
 *   1: the pair mass squared M^2 from a Breit-Wigner of (mz, wz) on the
 *      window [mlo^2, mhi^2] (arctangent map), then flat RAMBO over
 *      nfinal - 1 bodies (the pair as one particle of mass M first, the other
 *      finals in order), and an isotropic two-body decay of the pair in its
 *      rest frame;
 *   2: the same with M^2 distributed as 1/M^2 on the window (logarithmic map,
 *      the photon).
 * Each point's weight is 1 / sum_c alpha_c g_c(x), g_0 = 1 / V_n (V_n the
 * massless n-body volume) and, from the factorisation
 * dPhi_n = dPhi_{n-1} dM^2/(2 pi) dPhi_2 with Phi_2 = 1/(8 pi),
 * g_c = 2 pi p_c(M^2) / (w_R(x') Phi_2) for c = 1, 2 inside the window (0
 * outside), w_R(x') the massive RAMBO weight of the (n-1)-body configuration
 * (p_a + p_b, the others).  The weight is computed from the final momenta
 * alone, whichever channel made the point, so the sample estimates
 * integrals over flat phase space without bias (Kleiss, Pittau, Comput. Phys.
 * Commun. 83 (1994) 141).
 *
 * roots: sqrt(s) in GeV.  nfinal: 3..8.  pair_a, pair_b: final-state indices
 * (0-based, distinct) of the lepton pair.  mlo, mhi: the pair-mass window
 * (0 < mlo < mhi <= roots).  mz, wz: resonance mass and width (> 0).
 * alpha: host array of 3 channel weights (>= 0, positive sum).
 * seed, first_event: the Philox stream of ps_rambo; RAMBO particle i takes
 * uniforms 4i .. 4i + 3, uniform 32 picks the channel, 33 maps M^2, 34 and 35
 * give the decay angles (cos theta = 2u - 1, phi = 2 pi u').
 * momenta: device float64 [nevt][nfinal + 2][4], 16-byte aligned, layout of
 * ps_rambo.  weights: device float64 [nevt] or NULL.  channels: device int32
 * [nevt] or NULL, the channel that made each point.
 * Errors: ME_EINVAL (sizes, window, channel weights, alignment), ME_EDEVICE.
 */
int ps_multichannel(double roots, int nfinal, int pair_a, int pair_b, double mlo, double mhi, double mz, double wz,
                    const double *alpha, uint64_t seed, int64_t first_event, int64_t nevt, double *momenta,
                    double *weights, int32_t *channels, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PS_H */
