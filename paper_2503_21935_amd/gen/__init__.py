"""Process generator: Feynman diagrams, colour decomposition and HIP emission.

``generate(outdir)`` writes one header per process into ``outdir``.  It runs
at build time on the host; nothing here is imported on the GPU path at run
time except the static tables that ``info()`` reports.
"""
from __future__ import annotations

import os

from .coop import GGCoopEmitter
from .emit import GGEmitter
from .qew import QEWEmitter

GG_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
# Maximum number of wavefunctions kept alive at once by the emitted program
# (more are recomputed).  The momenta live in LDS, so the register budget
# goes to wavefunctions and J.  Chosen per process by compiling and timing:
# g g -> t tbar g g with every operand opaque ran fastest at 14 (49.5 ms per
# 2^20 events against 50.5 ms at 12, which has no private memory at all, and
# 44 bytes of it per lane at 14), with the polarisation-only copies at 13; g g -> t tbar g g g (workgroup program, J in LDS, window of 16)
# ran 334 ms per 2^18 events at 16 against 418 ms at 8 and 364 ms at 12 (18
# and 20 spill more and gain nothing); with the cache-aware amplitude order
# of the workgroup program it ran 304 ms at 16, and with opaque copies on the
# polarisations only (OPAQUE below) 299 ms at 12.
LIVE_CAP = {"gg_tt": 8, "gg_ttg": 8, "gg_ttgg": 13, "gg_ttggg": 12}
# the multi-channel programs (every operand opaque) keep the caps they were measured at
MC_LIVE_CAP = {"gg_tt": 8, "gg_ttg": 8, "gg_ttgg": 14}
LIVE_CAP_F32 = {"gg_tt": 8, "gg_ttg": 8, "gg_ttgg": 20, "gg_ttggg": 12}
# Processes whose colour-flow amplitudes are kept in LDS by a workgroup of
# waves sharing one program (see coop.py): register window of J per wave.
COOP_WINDOW = {"gg_ttggg": 16}
# Opaque operand copies (GGEmitter._opq): "eps" keeps them on the gluon
# polarisations only.  Measured per 2^20 events: g g -> t tbar g g 44.9 ms
# against 49.2 ms with every operand opaque, g ubar -> tau+ tau- g g ubar
# 8.8 ms against 9.5 ms; g g -> t tbar g g (with only the external
# spinors or only the internal currents opaque) 46.0 and 56.6 ms, and at cap
# 13 instead of 14 1 % faster again with 196 instead of 268 B/lane of private
# memory (45.8 against 46.5 ms at 8 helicity lanes on one box); g g -> t
# tbar g g g's workgroup program (with live-set cap 12 instead of 16) 299.4
# ms per 2^18 events against 305.4 ms.
OPAQUE = {"gg_tt": "eps", "gg_ttg": "eps", "gg_ttgg": "eps", "gg_ttggg": "eps"}
QEW_OPAQUE = "eps"
# Processes that also get the multi-channel program (single-diagram weights).
MULTICHANNEL = {"gg_tt", "gg_ttg", "gg_ttgg"}

# Quark-line + lepton-pair processes: n gluons, particle count, the quark
# line's row end (particle, 1 if an incoming antiquark vbar(p), 0 if an
# outgoing quark ubar(p)) and column end (particle, 1 if an incoming quark
# u(p), 0 if an outgoing antiquark v(p)), the l- and l+ particles, the gluons
# (particle, incoming), (charge, T3) of the quark and of the lepton, and the
# average over spins, colours and identical final states.  The momenta come
# in this particle order.
_UP, _TAU = (2.0 / 3.0, 0.5), (-1.0, -0.5)
QEW_SPECS = {
    "gux_taptamggux": dict(n=3, npart=7, row=(1, 1), col=(6, 0), lm=3, lp=2, gluons=((0, 1), (4, 0), (5, 0)),
                           quark=_UP, lepton=_TAU, avg=4 * 24 * 2, title="g ubar -> tau+ tau- g g ubar"),
    "gux_taptamgux": dict(n=2, npart=6, row=(1, 1), col=(5, 0), lm=3, lp=2, gluons=((0, 1), (4, 0)),
                          quark=_UP, lepton=_TAU, avg=4 * 24, title="g ubar -> tau+ tau- g ubar"),
    "gux_taptamux": dict(n=1, npart=5, row=(1, 1), col=(4, 0), lm=3, lp=2, gluons=((0, 1),),
                         quark=_UP, lepton=_TAU, avg=4 * 24, title="g ubar -> tau+ tau- ubar"),
}
# live-set caps of the quark-line programs (small: every program fits)
QEW_CAP = {"gux_taptamggux": 14, "gux_taptamgux": 12, "gux_taptamux": 12}


def generate(outdir: str, processes=None, merge: bool = True) -> dict:
    os.makedirs(outdir, exist_ok=True)
    info = {}
    for name, spec in QEW_SPECS.items():
        if processes and name not in processes:
            continue
        em = QEWEmitter(name, spec, merge=merge, cap=QEW_CAP[name], opaque=QEW_OPAQUE)
        src = em.render()
        path = os.path.join(outdir, f"proc_{name}.h")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)
        info[name] = dict(em.plan.stats(), lcd=em.lcd, ncol=len(em.perms))
    for name, n in GG_PROCESSES.items():
        if processes and name not in processes:
            continue
        if name in COOP_WINDOW:
            em = GGCoopEmitter(name, n, merge=merge, cap=LIVE_CAP[name], window=COOP_WINDOW[name],
                               opaque=OPAQUE[name])
        else:
            em = GGEmitter(name, n, merge=merge, cap=LIVE_CAP[name], cap_f32=LIVE_CAP_F32[name], opaque=OPAQUE[name])
        src = em.render()
        path = os.path.join(outdir, f"proc_{name}.h")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)
        info[name] = dict(em.plan.stats(), lcd=em.lcd, ncol=len(em.perms))
        if name in MULTICHANNEL:
            mc = GGEmitter(name, n, merge=False, cap=MC_LIVE_CAP[name])
            src = mc.render_mc()
            path = os.path.join(outdir, f"proc_{name}_mc.h")
            old = open(path).read() if os.path.exists(path) else None
            if old != src:
                with open(path, "w") as f:
                    f.write(src)
    return info
