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

#ifdef __cplusplus
}
#endif

#endif /* PS_H */
