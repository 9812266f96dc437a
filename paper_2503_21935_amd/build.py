"""Build libme.so for gfx950.

Steps: run the process generator into ``csrc/gen/``, write one translation
unit per process and the process table, compile each with hipcc
(``--offload-arch=gfx950``) and link the shared library in-tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libme.so")

PROCESSES = ["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gux_taptamux", "gux_taptamgux",
             "gux_taptamggux"]

# processes whose colour-flow amplitudes live in LDS (workgroup kernel of me_coop.h)
COOP = {"gg_ttggg"}

# one-wave processes that also get the float64 form with the colour sum on the
# matrix cores (needs a multiple of 4 colour flows); the workgroup processes
# always get it
CM = {"gg_ttgg"}

# Calibration of the mixed form's amplitude error estimate (multiplies
# u32 * 2 lambda_max(|N|) |S| |J| / Q); fixed by comparing float32 results
# with the oracle (see the mixed-precision tests).
MIXED_CEST = {"gg_tt": 8.0, "gg_ttg": 8.0, "gg_ttgg": 8.0, "gg_ttggg": 8.0}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-variable",
    "-Wno-unused-function", "-Wno-unknown-pragmas",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC,
]

_TU_QEW = """// Generated translation unit: kernels of {name} (quark line + lepton pair).
#include "me_qew.h"
{include}

static hipError_t launch_f64(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                             const me_params& prm, double* qhel, int lg, hipStream_t s) {{
    const dim3 grid((unsigned)(((nevt << lg) + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL((k_me_qew<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm, qhel,
                       nullptr, nullptr, lg);
    return hipGetLastError();
}}

static hipError_t launch_f64_idx(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                 const me_params& prm, const int* idx, const int* count, hipStream_t s) {{
    const dim3 grid((unsigned)((nevt + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL((k_me_qew<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm,
                       nullptr, idx, count, 0);
    return hipGetLastError();
}}

#ifndef __HIP_DEVICE_COMPILE__  // the table entry holds host function pointers
extern const me_process_desc me_desc_{name} = {{
    "{name}", ME_KIND_QEW, {proc}::npart, {proc}::ndiag, {proc}::ncol, {proc}::nhel,
    {proc}::flops_amp, {proc}::flops_colour, {proc}::flops_executed, launch_f64, launch_f64_idx, nullptr, 8.0,
    0.0, nullptr, nullptr, 0, nullptr}};
#endif
"""

_TU = """// Generated translation unit: kernels of {name}.
#include "me_mixed.h"
{include}

static hipError_t launch_f64(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                             const me_params& prm, double* qhel, int lg, hipStream_t s) {{
    const dim3 grid((unsigned)(((nevt << lg) + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL(({kernel}<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm,
                       qhel, nullptr, nullptr, lg);
    return hipGetLastError();
}}

static hipError_t launch_f64_idx(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                 const me_params& prm, const int* idx, const int* count, hipStream_t s) {{
    const dim3 grid((unsigned)((nevt + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL(({kernel}<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm,
                       nullptr, idx, count, 0);
    return hipGetLastError();
}}
{mixed}{cm}
#ifndef __HIP_DEVICE_COMPILE__  // the table entry holds host function pointers
extern const me_process_desc me_desc_{name} = {{
    "{name}", {kind}, {proc}::npart, {proc}::ndiag, {proc}::ncol, {proc}::nhel,
    {proc}::flops_amp, {proc}::flops_colour, {proc}::flops_executed, launch_f64, launch_f64_idx, {mixed_ptr}, {cest},
    {colerr}, {cm_ptr}, {mc_ptr}, {mc_n}, {mc_desc}}};
#endif
"""

_MC_DECL = """
#ifndef __HIP_DEVICE_COMPILE__
// the multi-channel kernel is compiled in a translation unit of its own
hipError_t me_launch_mc_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                               const me_params& prm, const int* chan, double* alpha, hipStream_t s);
extern const int me_nchan_{name};
extern const char* const* const me_chan_desc_{name};
#endif
"""

_TU_MC = """// Generated translation unit: multi-channel kernel of {name}.
#include "me_kernels.h"
#include "gen/proc_{name}_mc.h"

hipError_t me_launch_mc_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                               const me_params& prm, const int* chan, double* alpha, hipStream_t s) {{
    const dim3 grid((unsigned)((nevt + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL((k_me_gg_mc<proc_{name}_mc>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm,
                       chan, alpha);
    return hipGetLastError();
}}

#ifndef __HIP_DEVICE_COMPILE__
extern const int me_nchan_{name} = proc_{name}_mc::nchan;
extern const char* const* const me_chan_desc_{name} = channel_desc_{name};
#endif
"""

_CM = """
static hipError_t launch_f64_cm(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                const me_params& prm, double* qhel, int lg, hipStream_t s) {{
    const dim3 grid((unsigned)(((nevt << lg) + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL((k_me_gg_cm<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm, qhel,
                       nullptr, nullptr, lg);
    return hipGetLastError();
}}
"""

_TU_COOP = """// Generated translation unit: kernels of {name} (workgroup form, J in LDS).
#include "me_coop.h"
{include}

static hipError_t launch_f64(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                             const me_params& prm, double* qhel, int lg, hipStream_t s) {{
    const dim3 grid((unsigned)(((nevt << lg) + ME_TILE - 1) / ME_TILE));
    hipLaunchKernelGGL((k_me_gg_coop<{proc}>), grid, dim3(ME_TILE * {proc}::waves), 0, s, mom, nevt, out, hels,
                       nh, prm, qhel, nullptr, nullptr, lg);
    return hipGetLastError();
}}

static hipError_t launch_f64_idx(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                 const me_params& prm, const int* idx, const int* count, hipStream_t s) {{
    const dim3 grid((unsigned)((nevt + ME_TILE - 1) / ME_TILE));
    hipLaunchKernelGGL((k_me_gg_coop<{proc}>), grid, dim3(ME_TILE * {proc}::waves), 0, s, mom, nevt, out, hels,
                       nh, prm, nullptr, idx, count, 0);
    return hipGetLastError();
}}

#ifndef __HIP_DEVICE_COMPILE__  // the table entry holds host function pointers
// the mixed-precision launcher and the matrix-core colour form are compiled in
// translation units of their own
hipError_t me_launch_mixed_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                  const me_params& prm, float tol, float cest, int* flag_count, int* flag_idx,
                                  float* err_out, unsigned char* flag_out, hipStream_t s);
hipError_t me_launch_f64_cm_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                   const me_params& prm, double* qhel, int lg, hipStream_t s);
extern const me_process_desc me_desc_{name} = {{
    "{name}", ME_KIND_GG, {proc}::npart, {proc}::ndiag, {proc}::ncol, {proc}::nhel,
    {proc}::flops_amp, {proc}::flops_colour, {proc}::flops_executed, launch_f64, launch_f64_idx, me_launch_mixed_{name}, {cest},
    {proc}::colour_err_f16, me_launch_f64_cm_{name}, nullptr, 0, nullptr}};
#endif
"""

_TU_COOP_CM = """// Generated translation unit: float64 kernel of {name} with the colour sum on the matrix cores.
#include "me_coop.h"
{include}

hipError_t me_launch_f64_cm_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                   const me_params& prm, double* qhel, int lg, hipStream_t s) {{
    const dim3 grid((unsigned)(((nevt << lg) + ME_TILE - 1) / ME_TILE));
    hipLaunchKernelGGL((k_me_gg_coop<{proc}, true>), grid, dim3(ME_TILE * {proc}::waves), 0, s, mom, nevt, out,
                       hels, nh, prm, qhel, nullptr, nullptr, lg);
    return hipGetLastError();
}}
"""

_TU_COOP_MIXED = """// Generated translation unit: mixed-precision kernel of {name} (workgroup form).
#include "me_coop_mixed.h"
{include}

hipError_t me_launch_mixed_{name}(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                                  const me_params& prm, float tol, float cest, int* flag_count, int* flag_idx,
                                  float* err_out, unsigned char* flag_out, hipStream_t s) {{
    if (flag_count) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, flag_count);
    const dim3 grid((unsigned)((nevt + ME_TILE - 1) / ME_TILE));
    hipLaunchKernelGGL((k_me_gg_coop_mixed<{proc}>), grid, dim3(ME_TILE * {proc}::waves), 0, s, mom, nevt, out,
                       hels, nh, prm, tol, cest, flag_count, flag_idx, err_out, flag_out);
    return hipGetLastError();
}}
"""

_MIXED = """
static hipError_t launch_mixed(const double* mom, int64_t nevt, double* out, const int* hels, int nh,
                               const me_params& prm, float tol, float cest, int* flag_count, int* flag_idx,
                               float* err_out, unsigned char* flag_out, hipStream_t s) {{
    if (flag_count) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, flag_count);
    const dim3 grid((unsigned)((nevt + ME_BLOCK - 1) / ME_BLOCK));
    hipLaunchKernelGGL((k_me_gg_mixed<{proc}>), grid, dim3(ME_BLOCK), 0, s, mom, nevt, out, hels, nh, prm, tol,
                       cest, flag_count, flag_idx, err_out, flag_out);
    return hipGetLastError();
}}
"""

_REG = """// Generated process table.
#include <cstring>
#include "me_launch.h"
{decls}
static const me_process_desc* const table[] = {{{ptrs}}};

const me_process_desc* me_find_process(const char* name) {{
    for (const me_process_desc* d : table)
        if (std::strcmp(d->name, name) == 0) return d;
    return nullptr;
}}
"""


def _write(path, text):
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)


def generate_sources(processes):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2503_21935_amd.gen import MULTICHANNEL, QEW_SPECS, generate

    info = generate(GEN, [p for p in processes if p.startswith("gg_") or p in QEW_SPECS])
    tus = []
    for name in processes:
        if name in QEW_SPECS:
            path = os.path.join(GEN, f"tu_{name}.hip")
            _write(path, _TU_QEW.format(name=name, include=f'#include "gen/proc_{name}.h"', proc=f"proc_{name}"))
            tus.append(path)
            continue
        if name == "ee_mumu":
            inc, kernel, proc, kind = "", "k_me_ee", "proc_ee_mumu", "ME_KIND_EE"
            mixed, mixed_ptr, colerr = "", "nullptr", "0.0"
        else:
            inc, kernel, proc, kind = f'#include "gen/proc_{name}.h"', "k_me_gg", f"proc_{name}", "ME_KIND_GG"
            mixed, mixed_ptr, colerr = _MIXED.format(proc=proc), "launch_mixed", f"{proc}::colour_err_f16"
        path = os.path.join(GEN, f"tu_{name}.hip")
        if name in COOP:
            _write(path, _TU_COOP.format(name=name, include=inc, proc=proc, cest=MIXED_CEST.get(name, 8.0)))
            tus.append(path)
            path_m = os.path.join(GEN, f"tu_{name}_mixed.hip")
            _write(path_m, _TU_COOP_MIXED.format(name=name, include=inc, proc=proc))
            tus.append(path_m)
            path_c = os.path.join(GEN, f"tu_{name}_cm.hip")
            _write(path_c, _TU_COOP_CM.format(name=name, include=inc, proc=proc))
            tus.append(path_c)
            continue
        cm, cm_ptr = ("", "nullptr")
        if name in CM:
            cm, cm_ptr = _CM.format(proc=proc), "launch_f64_cm"
        mc_ptr, mc_n, mc_desc = "nullptr", "0", "nullptr"
        if name in MULTICHANNEL:
            cm += _MC_DECL.format(name=name)
            mc_ptr, mc_n, mc_desc = f"me_launch_mc_{name}", f"me_nchan_{name}", f"me_chan_desc_{name}"
            path_mc = os.path.join(GEN, f"tu_{name}_mc.hip")
            _write(path_mc, _TU_MC.format(name=name))
            tus.append(path_mc)
        _write(path, _TU.format(name=name, include=inc, kernel=kernel, proc=proc, kind=kind, mixed=mixed,
                                mixed_ptr=mixed_ptr, cest=MIXED_CEST.get(name, 8.0), colerr=colerr, cm=cm,
                                cm_ptr=cm_ptr, mc_ptr=mc_ptr, mc_n=mc_n, mc_desc=mc_desc))
        tus.append(path)
    decls = "\n".join(f"extern const me_process_desc me_desc_{n};" for n in processes)
    ptrs = ", ".join(f"&me_desc_{n}" for n in processes)
    reg = os.path.join(GEN, "registry.cpp")
    _write(reg, _REG.format(decls=decls, ptrs=ptrs))
    return tus + [reg, os.path.join(CSRC, "me_api.cpp"), os.path.join(CSRC, "mlp.hip"),
                  os.path.join(CSRC, "me_unweight.hip"), os.path.join(CSRC, "ps_rambo.hip")], info


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC] + HIPFLAGS + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def build(processes=None, jobs: int = 8, verbose: bool = True):
    processes = processes or PROCESSES
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    srcs, info = generate_sources(processes)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return info


if __name__ == "__main__":
    procs = sys.argv[1:] or None
    build(procs)
