"""CPU oracle for the per-event squared matrix element (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg, never by the product path.  It shares
no code with the HIP library (``paper_2503_21935_amd``) and neither imports
the other; both read momenta from the separate ``inputs`` module.

Contents
  * ``sm_params``      derived Standard-Model constants for the workloads
  * ``colour_matrix``  C_kl = sum over colours of conj(c_k) c_l, by definition,
                        with explicit Gell-Mann matrices
  * ``me2``            |M|^2 per event (C routines in ``me_oracle.c``)
  * ``ordered_amps``   colour-ordered partial amplitudes at one helicity
  * ``me2_dressed``    |M|^2 by explicit colour brute force (slow; few events)
  * ``channel_diagrams``, ``diagram_sums``  single Feynman diagrams (route 4)
  * ``rambo``, ``ps_mc``  phase-space points: flat RAMBO, and multi-channel
                        sampling of a final state with a lepton pair (ps_oracle.c)
  * ``qew_me2``, ``qew_amps``  a massless quark line with gluons and a photon/Z
                        decaying to leptons (route 5; QEW_PROCESSES, among
                        them the paper's DY+3j subprocess g ubar -> tau+ tau- g g ubar)

The paper gives no formulas; the matrix element is the textbook tree-level one
(its Sec. 2 names the step, Sec. 3 the two parts -- Feynman diagrams, then the
colour-matrix quadratic form).  Parameter readings: electroweak inputs
(alpha, G_F, M_Z), so M_W and sin^2(theta_W) are derived; fixed widths;
T^a = lambda^a / 2; normalisation 1/(spins x colours x identical finals).
"""
from __future__ import annotations

import ctypes
import functools
import itertools
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "me_oracle.c")
_LIBS = {False: os.path.join(_HERE, "liboracle.so"), True: os.path.join(_HERE, "liboracle_quad.so")}
_PS_SRC = os.path.join(_HERE, "ps_oracle.c")
_PS_LIB = os.path.join(_HERE, "liboracle_ps.so")

PROCESS_NGLUON = {"gg_tt": 2, "gg_ttg": 3, "gg_ttgg": 4, "gg_ttggg": 5}


def _build_ps(force: bool = True) -> None:
    if not force and os.path.exists(_PS_LIB) and os.path.getmtime(_PS_LIB) >= os.path.getmtime(_PS_SRC):
        return
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", _PS_LIB + ".tmp", _PS_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_PS_LIB + ".tmp", _PS_LIB)


def build(force: bool = True) -> None:
    """Compile the double and __float128 variants of the matrix-element oracle
    and the phase-space oracle with gcc."""
    _build_ps(force)
    for quad, lib in _LIBS.items():
        if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", lib + ".tmp", _SRC]
        if quad:
            cmd[1:1] = ["-DORACLE_QUAD"]
            cmd += ["-lquadmath"]
        cmd += ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)


@functools.lru_cache(maxsize=None)
def _lib(quad: bool = False):
    path = _LIBS[quad]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=False)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_ee_mumu.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, dp, dp]
    lib.oracle_ggx.argtypes = [dp, ctypes.c_int64, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, dp, dp]
    lib.oracle_ggx_amps.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
    lib.oracle_ggx_diagram_amps.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, dp]
    lib.oracle_ggx_diagrams.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, dp]
    lib.oracle_ggx_dressed.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       dp, dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_qew.argtypes = [dp, ctypes.c_int64, ip, dp, dp, ctypes.c_double, dp, dp]
    lib.oracle_qew_amps.argtypes = [dp, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_qew_externals.argtypes = [dp, ip, dp, ctypes.c_int, dp]
    lib.oracle_bg_custom.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ip, ctypes.c_int, dp]
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------

def sm_params(alpha_s=0.118, inv_alpha=132.507, gf=1.16639e-5, mz=91.188, wz=2.4414, mt=173.0, wt=1.4915):
    """Derived couplings.  M_W from (alpha, G_F, M_Z):
    M_W^2 = M_Z^2/2 + sqrt(M_Z^4/4 - pi alpha M_Z^2 / (sqrt2 G_F))."""
    alpha = 1.0 / inv_alpha
    mw = math.sqrt(mz ** 2 / 2 + math.sqrt(mz ** 4 / 4 - math.pi * alpha * mz ** 2 / (math.sqrt(2) * gf)))
    sw2 = 1 - mw ** 2 / mz ** 2
    return dict(e=math.sqrt(4 * math.pi * alpha), gs=math.sqrt(4 * math.pi * alpha_s), sw2=sw2, mw=mw,
                mz=mz, wz=wz, mt=mt, wt=wt)


# --------------------------------------------------------------------------
# Colour
# --------------------------------------------------------------------------

def gell_mann() -> np.ndarray:
    """T^a = lambda^a / 2, shape [8][3][3]."""
    l = np.zeros((8, 3, 3), dtype=complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7] = np.diag([1, 1, -2]) / math.sqrt(3)
    return l / 2


def orderings(n: int):
    """Gluon orderings in the order the oracle and its colour matrix use
    (lexicographic permutations of gluon labels 0..n-1)."""
    return list(itertools.permutations(range(n)))


@functools.lru_cache(maxsize=None)
def colour_matrix(n: int) -> np.ndarray:
    """C_kl = sum_{a_1..a_n, i, j} conj(c_k) c_l with c_k = (T^{a_s1} ... T^{a_sn})_{ij},
    s = orderings(n)[k]: the plain definition, summed with Gell-Mann matrices."""
    T = gell_mann()
    # W[a_1, ..., a_n, i, j] = (T^{a_1} ... T^{a_n})_{ij}
    W = T
    for _ in range(n - 1):
        W = np.einsum("...ij,bjk->...bik", W, T)
    perms = orderings(n)
    # c_sigma(a)_{ij} = W[a_{sigma1}, ..., a_{sigma n}]_{ij}; as an array over a this is
    # W with axis sigma_m moved to position m.
    rows = []
    for s in perms:
        inv = np.argsort(s)
        rows.append(np.transpose(W, tuple(inv) + (n, n + 1)).reshape(-1))
    V = np.stack(rows)
    C = (V.conj() @ V.T).real
    return C


# --------------------------------------------------------------------------
# Matrix elements
# --------------------------------------------------------------------------

def _check_mom(mom, npart):
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    if mom.ndim != 3 or mom.shape[1:] != (npart, 4):
        raise ValueError(f"momenta must be [nevt][{npart}][4], got {mom.shape}")
    return mom


def me2(process: str, mom, params=None, quad: bool = False, per_helicity: bool = False):
    """Spin- and colour-summed/averaged |M|^2 for every event in ``mom``."""
    p = params or sm_params()
    lib = _lib(quad)
    if process == "ee_mumu":
        mom = _check_mom(mom, 4)
        n = mom.shape[0]
        out = np.empty(n)
        qh = np.empty((n, 16)) if per_helicity else None
        rc = lib.oracle_ee_mumu(_ptr(mom), n, p["e"], p["sw2"], p["mz"], p["wz"], _ptr(out), _ptr(qh))
    elif process in QEW_PROCESSES:
        return qew_me2(process, mom, params, quad=quad, per_helicity=per_helicity)
    elif process in PROCESS_NGLUON:
        ng = PROCESS_NGLUON[process]
        mom = _check_mom(mom, ng + 2)
        n = mom.shape[0]
        C = np.ascontiguousarray(colour_matrix(ng))
        out = np.empty(n)
        qh = np.empty((n, 1 << (ng + 2))) if per_helicity else None
        rc = lib.oracle_ggx(_ptr(mom), n, ng, _ptr(C), p["gs"], p["mt"], p["wt"], _ptr(out), _ptr(qh))
    else:
        raise KeyError(process)
    if rc != 0:
        raise RuntimeError(f"oracle failed ({rc})")
    return (out, qh) if per_helicity else out


def ordered_amps(n: int, mom1, hel: int, params=None, gauge_gluon: int = -1, quad: bool = False,
                 four_gluon: bool = True):
    """Colour-ordered partial amplitudes J[k] (k over ``orderings(n)``) of one event.
    four_gluon=False leaves the four-gluon vertex out of the recursion: the sum
    over the ordered diagrams built from three-point vertices only."""
    p = params or sm_params()
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64).reshape(n + 2, 4)
    out = np.empty((math.factorial(n), 2))
    rc = _lib(quad).oracle_ggx_amps(_ptr(mom1), n, hel, gauge_gluon, p["gs"], p["mt"], p["wt"], _ptr(out),
                                    int(four_gluon))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return out[:, 0] + 1j * out[:, 1]


def me2_dressed(n: int, mom1, params=None, per_helicity: bool = False):
    """|M|^2 of one event by explicit colour brute force (n <= 4 gluons)."""
    p = params or sm_params()
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64).reshape(n + 2, 4)
    out = np.empty(1)
    qh = np.empty(1 << (n + 2))
    rc = _lib(False).oracle_ggx_dressed(_ptr(mom1), n, p["gs"], p["mt"], p["wt"], _ptr(out), _ptr(qh))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return (out[0], qh) if per_helicity else out[0]


# --------------------------------------------------------------------------
# Single Feynman diagrams (route 4): the multi-channel weights
# --------------------------------------------------------------------------

_MAXG = 5
_DIAG_STRIDE = 2 + _MAXG + 3 * 2 * _MAXG


def _trees(S):
    """Binary gluon trees over the set S (three-gluon vertices only), as nested
    tuples; the subtree holding the smallest label comes first."""
    S = tuple(sorted(S))
    if len(S) == 1:
        return [S[0]]
    first, rest = S[0], S[1:]
    out = []
    for k in range(0, len(rest)):
        for extra in itertools.combinations(rest, k):
            A = (first,) + extra
            B = tuple(x for x in rest if x not in extra)
            if not B:
                continue
            for ta in _trees(A):
                for tb in _trees(B):
                    out.append((ta, tb))
    return out


def _ordered_set_partitions(items):
    items = tuple(items)
    if not items:
        yield ()
        return
    for k in range(1, len(items) + 1):
        for first in itertools.combinations(items, k):
            rest = tuple(x for x in items if x not in first)
            for tail in _ordered_set_partitions(rest):
                yield (first,) + tail


def _tree_desc(t):
    if isinstance(t, int):
        return str(t)
    return "(" + _tree_desc(t[0]) + "," + _tree_desc(t[1]) + ")"


def channel_diagrams(n: int):
    """Every Feynman diagram of g g -> t tbar + (n-2) g whose gluons meet only
    at three-point vertices: the channels of the multi-channel weights.  A
    diagram is a sequence of gluon trees attached along the top line from
    ubar(p3) to v(p4).  Returns (descriptors, encoding [ndiag][stride] int32);
    a descriptor writes the trees in top-line order separated by '|', a tree
    as nested '(x,y)' with the part holding the smaller label first."""
    descs, rows = [], []
    for part in _ordered_set_partitions(range(n)):
        for trees in itertools.product(*(_trees(B) for B in part)):
            nodes, roots = [], []

            def emit(t):
                if isinstance(t, int):
                    nodes.append((-1, -1, t))
                else:
                    l = emit(t[0])
                    r = emit(t[1])
                    nodes.append((l, r, -1))
                return len(nodes) - 1

            for t in trees:
                roots.append(emit(t))
            row = np.zeros(_DIAG_STRIDE, dtype=np.int32)
            row[0] = len(roots)
            row[1:1 + len(roots)] = roots
            row[1 + _MAXG] = len(nodes)
            for i, (l, r, leaf) in enumerate(nodes):
                row[2 + _MAXG + 3 * i: 2 + _MAXG + 3 * i + 3] = (l, r, leaf)
            rows.append(row)
            descs.append("|".join(_tree_desc(t) for t in trees))
    return descs, np.stack(rows)


def diagram_amps(n: int, mom1, hel: int, params=None):
    """Complex amplitudes A_d of every channel diagram (order of
    channel_diagrams) of one event at one helicity."""
    p = params or sm_params()
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64).reshape(n + 2, 4)
    descs, enc = channel_diagrams(n)
    enc = np.ascontiguousarray(enc)
    out = np.empty((len(descs), 2))
    rc = _lib(False).oracle_ggx_diagram_amps(_ptr(mom1), n, hel, len(descs),
                                             enc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), p["gs"], p["mt"],
                                             p["wt"], _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return descs, out[:, 0] + 1j * out[:, 1]


def diagram_sums(process: str, mom, params=None):
    """sum over all helicities of |A_d|^2 for every channel diagram d of the
    process (order of channel_diagrams), per event: [nevt][ndiag]."""
    p = params or sm_params()
    ng = PROCESS_NGLUON[process]
    mom = _check_mom(mom, ng + 2)
    descs, enc = channel_diagrams(ng)
    enc = np.ascontiguousarray(enc)
    out = np.empty((mom.shape[0], len(descs)))
    lib = _lib(False)
    rc = lib.oracle_ggx_diagrams(_ptr(mom), mom.shape[0], ng, len(descs),
                                 enc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), p["gs"], p["mt"], p["wt"],
                                 _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return descs, out


# --------------------------------------------------------------------------
# Phase-space sampling (ps_oracle.c): Philox4x32-10 and RAMBO
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def _ps_lib():
    _build_ps(force=False)
    lib = ctypes.CDLL(_PS_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_philox4x32.argtypes = [u32p, u32p, ctypes.c_int, u32p]
    lib.oracle_event_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, dp]
    lib.oracle_rambo.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, dp, dp, dp]
    lib.oracle_ps_mc.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.POINTER(ctypes.c_int32), dp]
    return lib


def philox4x32(ctr, key, rounds: int = 10):
    """Philox4x32 block function (Salmon et al., SC'11): four 32-bit words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    _ps_lib().oracle_philox4x32(c, k, int(rounds), o)
    return [int(v) for v in o]


def event_uniforms(seed: int, event: int, n: int) -> np.ndarray:
    """The n uniforms of one event of the phase-space stream."""
    out = np.empty(n)
    _ps_lib().oracle_event_uniforms(int(seed), int(event), int(n), _ptr(out))
    return out


def rambo(roots: float, masses, seed: int, first: int, n_evt: int, cond: bool = False):
    """Flat phase-space points (momenta [n][nf + 2][4], weights [n]) of events
    first .. first + n_evt - 1 of the Philox stream `seed` (RAMBO map); with
    cond=True also the per-event factor (Q0/M)^2 by which the map enlarges
    rounding in the generated directions and energies."""
    m = np.ascontiguousarray(masses, dtype=np.float64)
    nf = m.size
    mom = np.empty((n_evt, nf + 2, 4))
    wt = np.empty(n_evt)
    cd = np.empty(n_evt) if cond else None
    rc = _ps_lib().oracle_rambo(float(roots), _ptr(m), nf, int(seed), int(first), int(n_evt), _ptr(mom), _ptr(wt),
                                _ptr(cd))
    if rc != 0:
        raise ValueError("oracle_rambo: bad arguments")
    return (mom, wt, cd) if cond else (mom, wt)


def ps_mc(roots: float, n: int, pair, window, mz: float, wz: float, alpha, seed: int, first: int, n_evt: int):
    """Multi-channel points (flat RAMBO, a Z Breit-Wigner and a photon 1/M^2
    channel on the invariant mass of the final-state pair (a, b), massless
    finals): momenta [n_evt][n + 2][4], multi-channel weights, the channel of
    each point and the weight its channel alone gives it."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    mom = np.empty((n_evt, n + 2, 4))
    wt = np.empty(n_evt)
    ch = np.empty(n_evt, dtype=np.int32)
    wc = np.empty(n_evt)
    rc = _ps_lib().oracle_ps_mc(float(roots), int(n), int(pair[0]), int(pair[1]), float(window[0]),
                                float(window[1]), float(mz), float(wz), _ptr(a), int(seed), int(first), int(n_evt),
                                _ptr(mom), _ptr(wt), ch.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(wc))
    if rc != 0:
        raise ValueError("oracle_ps_mc: bad arguments")
    return mom, wt, ch, wc


# --------------------------------------------------------------------------
# Route 5: one massless quark line, gluons and gamma/Z -> lepton pair
# --------------------------------------------------------------------------

_QEW_DESC = 8 + 2 * _MAXG

# n gluons, particle count, row end (particle, kind: 0 outgoing quark ubar(p),
# 1 incoming antiquark vbar(p)), column end (particle, kind: 0 outgoing
# antiquark v(p), 1 incoming quark u(p)), lepton l- and l+ particles, gluons
# (particle, incoming), (Q, T3) of the quark line and of the leptons, and the
# average: spins x colours x identical final-state factor.
QEW_PROCESSES = {
    # g ubar -> tau+ tau- g g ubar: the paper's DY+3j subprocess (Sec. 3)
    "gux_taptamggux": dict(n=3, npart=7, row=(1, 1), col=(6, 0), lm=3, lp=2, gluons=((0, 1), (4, 0), (5, 0)),
                           quark=(2.0 / 3.0, 0.5), lepton=(-1.0, -0.5), avg=4 * 24 * 2),
    # the same family with fewer gluons
    "gux_taptamgux": dict(n=2, npart=6, row=(1, 1), col=(5, 0), lm=3, lp=2, gluons=((0, 1), (4, 0)),
                          quark=(2.0 / 3.0, 0.5), lepton=(-1.0, -0.5), avg=4 * 24),
    "gux_taptamux": dict(n=1, npart=5, row=(1, 1), col=(4, 0), lm=3, lp=2, gluons=((0, 1),),
                         quark=(2.0 / 3.0, 0.5), lepton=(-1.0, -0.5), avg=4 * 24),
    # u ubar -> tau+ tau-: lowest-order Drell-Yan
    "uux_taptam": dict(n=0, npart=4, row=(1, 1), col=(0, 1), lm=3, lp=2, gluons=(),
                       quark=(2.0 / 3.0, 0.5), lepton=(-1.0, -0.5), avg=4 * 9),
}


def _qew_spec(process):
    return QEW_PROCESSES[process] if isinstance(process, str) else process


def _qew_arrays(spec, params):
    p = params or sm_params()
    desc = np.zeros(_QEW_DESC, dtype=np.int32)
    desc[:8] = [spec["n"], spec["npart"], spec["row"][0], spec["row"][1], spec["col"][0], spec["col"][1],
                spec["lm"], spec["lp"]]
    for a, (pi, inc) in enumerate(spec["gluons"]):
        desc[8 + a] = pi
        desc[8 + _MAXG + a] = inc
    cpl = np.array([p["e"], p["sw2"], p["mz"], p["wz"], p["gs"], *spec["quark"], *spec["lepton"]],
                   dtype=np.float64)
    return desc, cpl


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def qew_colour(n: int) -> np.ndarray:
    """Colour matrix of a quark line with n gluons (n = 0: sum_ij delta_ij delta_ij = 3)."""
    return np.array([[3.0]]) if n == 0 else np.ascontiguousarray(colour_matrix(n))


def qew_me2(process, mom, params=None, quad: bool = False, per_helicity: bool = False, colour=None):
    """|M|^2 per event for a quark line with gluons and a gamma/Z -> lepton pair
    (``process`` a name in QEW_PROCESSES or a spec of the same form)."""
    spec = _qew_spec(process)
    desc, cpl = _qew_arrays(spec, params)
    mom = _check_mom(mom, spec["npart"])
    n = mom.shape[0]
    C = np.ascontiguousarray(qew_colour(spec["n"]) if colour is None else colour, dtype=np.float64)
    out = np.empty(n)
    qh = np.empty((n, 1 << spec["npart"])) if per_helicity else None
    rc = _lib(quad).oracle_qew(_ptr(mom), n, _ip(desc), _ptr(cpl), _ptr(C), 1.0 / spec["avg"], _ptr(out), _ptr(qh))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return (out, qh) if per_helicity else out


def qew_amps(process, mom1, hel: int, params=None, gauge_gluon: int = -1, gauge_ew: bool = False,
             quad: bool = False):
    """Colour-ordered partial amplitudes (orders of ``orderings(n)``) of one event at one helicity."""
    spec = _qew_spec(process)
    desc, cpl = _qew_arrays(spec, params)
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64).reshape(spec["npart"], 4)
    out = np.empty((math.factorial(spec["n"]), 2))
    rc = _lib(quad).oracle_qew_amps(_ptr(mom1), _ip(desc), _ptr(cpl), hel, gauge_gluon, int(gauge_ew), _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return out[:, 0] + 1j * out[:, 1]


def qew_externals(process, mom1, hel: int, params=None):
    """External pieces of one event at one helicity: dict of gluon q and eps, the
    row spinor and its momentum, the column spinor, the insertion's momentum qE
    and vectors EL, ER (couplings and propagators included)."""
    spec = _qew_spec(process)
    desc, cpl = _qew_arrays(spec, params)
    n = spec["n"]
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64).reshape(spec["npart"], 4)
    out = np.empty(4 * n + 8 * n + 4 + 8 + 8 + 4 + 8 + 8)
    rc = _lib(False).oracle_qew_externals(_ptr(mom1), _ip(desc), _ptr(cpl), hel, _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle failed")
    o = 0

    def take(k):
        nonlocal o
        v = out[o:o + k]
        o += k
        return v

    q = take(4 * n).reshape(n, 4)
    eps = take(8 * n).reshape(n, 4, 2)
    prow = take(4)
    row = take(8).reshape(4, 2)
    col = take(8).reshape(4, 2)
    qE = take(4)
    EL = take(8).reshape(4, 2)
    ER = take(8).reshape(4, 2)
    c = lambda a: a[..., 0] + 1j * a[..., 1]  # noqa: E731
    return dict(q=q, eps=c(eps), prow=prow, row=c(row), col=c(col), qE=qE, EL=c(EL), ER=c(ER))


def bg_custom(q, eps, prow, row, col, sigma, g, m=0.0, w=0.0, four_gluon: bool = True):
    """Route 2's colour-ordered amplitude (quark line with gluon-like legs) for
    explicit externals: q [n][4] incoming-flow momenta, eps [n][4] complex
    vectors, the row spinor with its momentum, the column spinor; one order."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0]
    e = np.ascontiguousarray(np.stack([np.real(eps), np.imag(eps)], axis=-1), dtype=np.float64)
    r = np.ascontiguousarray(np.stack([np.real(row), np.imag(row)], axis=-1), dtype=np.float64)
    c = np.ascontiguousarray(np.stack([np.real(col), np.imag(col)], axis=-1), dtype=np.float64)
    pr = np.ascontiguousarray(prow, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.int32)
    out = np.empty(2)
    rc = _lib(False).oracle_bg_custom(n, _ptr(q), _ptr(e), _ptr(pr), _ptr(r), _ptr(c), m, w, g, _ip(s),
                                      int(four_gluon), _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle failed")
    return out[0] + 1j * out[1]
