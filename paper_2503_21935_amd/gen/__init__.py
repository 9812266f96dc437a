"""Process generator: Feynman diagrams, colour decomposition and HIP emission.

``generate(outdir)`` writes one header per process into ``outdir``.  It runs
at build time on the host; nothing here is imported on the GPU path at run
time except the static tables that ``info()`` reports.
"""
from __future__ import annotations

import os

from .coop import GGCoopEmitter
from .emit import GGEmitter

GG_PROCESSES = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}
# Maximum number of wavefunctions kept alive at once by the emitted program
# (more are recomputed).  Chosen per process by compiling and counting
# float64 operations plus VGPR<->AGPR moves (both take a VALU issue slot):
# g g -> t tbar g g is cheapest at 10 without scratch spills (12 and above
# spill); the float32 program fits without any recomputation.  For
# g g -> t tbar g g g (workgroup program, no J in registers) 8 with a window of
# 16 leaves the least private memory.
LIVE_CAP = {"gg_tt": 8, "gg_ttg": 8, "gg_ttgg": 10, "gg_ttggg": 8}
LIVE_CAP_F32 = {"gg_tt": 8, "gg_ttg": 8, "gg_ttgg": 20, "gg_ttggg": 12}
# Processes whose colour-flow amplitudes are kept in LDS by a workgroup of
# waves sharing one program (see coop.py): register window of J per wave.
COOP_WINDOW = {"gg_ttggg": 16}


def generate(outdir: str, processes=None, merge: bool = True) -> dict:
    os.makedirs(outdir, exist_ok=True)
    info = {}
    for name, n in GG_PROCESSES.items():
        if processes and name not in processes:
            continue
        if name in COOP_WINDOW:
            em = GGCoopEmitter(name, n, merge=merge, cap=LIVE_CAP[name], window=COOP_WINDOW[name])
        else:
            em = GGEmitter(name, n, merge=merge, cap=LIVE_CAP[name], cap_f32=LIVE_CAP_F32[name])
        src = em.render()
        path = os.path.join(outdir, f"proc_{name}.h")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)
        info[name] = dict(em.plan.stats(), lcd=em.lcd, ncol=len(em.perms))
    return info
