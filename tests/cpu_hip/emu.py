"""CPU build of librmx (host core + HIP kernels) over a host emulation of HIP, for
running the kernels' logic under AddressSanitizer on tiny inputs.  Test infrastructure
only: the product path never loads it."""
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2104_00095_amd", "csrc")
EXE = os.path.join(HERE, "run_case_emu")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SOURCES = [os.path.join(CSRC, f) for f in
           ("rmx_kernels.hip", "rmx_plan.cpp", "rmx_core.cpp", "rmx_server.cpp")] + \
          [os.path.join(HERE, "hip_emu.cpp"), os.path.join(HERE, "run_case.cpp")]


def build(sanitize=True):
    srcs = SOURCES
    newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(HERE, "hip", "hip_runtime.h")]
                 + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")])
    if os.path.exists(EXE) and os.path.getmtime(EXE) > newest:
        return EXE
    flags = ["-std=c++20", "-g", "-O1", "-fno-omit-frame-pointer", "-Wno-unknown-attributes",
             "-Wno-unused-command-line-argument", "-I", HERE, "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-DRMX_EMU_REDZONES"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = [CLANG] + flags + ["-x", "c++"] + srcs + ["-o", EXE + ".tmp", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(EXE + ".tmp", EXE)
    return EXE


def run(w, tmpdir, r_s=2, r_max=4, normal_layers=2, precision=0, flags=0, reps=1,
        xi_normal=None, timeout=600, pre_flags=(), cus=None):
    """Write workload `w` to tmpdir, run the emulated library, return
    (status, [(xi_out, labels, decisions, stats_raw)])."""
    os.makedirs(tmpdir, exist_ok=True)
    lines = [f"{len(w.solids)} {w.grid_n[0]} {w.grid_n[1]} {w.grid_n[2]} {w.h!r} "
             f"{w.origin[0]!r} {w.origin[1]!r} {w.origin[2]!r}",
             f"{r_s} {r_max} {normal_layers} {precision} {flags} {reps}"]
    for i, s in enumerate(w.solids):
        sh = s.shape
        has_n = xi_normal is not None and xi_normal[i] is not None
        vals = list(s.lo) + list(s.ext) + [s.n_layers, sh.kind]
        fl = list(map(float, sh.centre)) + list(map(float, sh.semi)) + \
            list(map(float, np.asarray(sh.rot).reshape(-1)))
        lines.append(" ".join(str(int(v)) for v in vals) + " " +
                     " ".join(repr(v) for v in fl) + f" {int(has_n)}")
        np.ascontiguousarray(s.xi, dtype=np.float64).tofile(os.path.join(tmpdir, f"xi{i}.bin"))
        if has_n:
            np.ascontiguousarray(xi_normal[i], dtype=np.float64).tofile(
                os.path.join(tmpdir, f"xn{i}.bin"))
    with open(os.path.join(tmpdir, "case.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    pre = os.path.join(tmpdir, "pre_flags.txt")
    if pre_flags:
        with open(pre, "w") as f:
            f.write(" ".join(str(int(v)) for v in pre_flags) + "\n")
    elif os.path.exists(pre):
        os.remove(pre)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    if cus is not None:   # compute units the emulated device reports
        env["RMX_EMU_CUS"] = str(int(cus))
    subprocess.run([build(), tmpdir], check=True, timeout=timeout, env=env)
    st = int(open(os.path.join(tmpdir, "status.txt")).read())
    outs = []
    for i, s in enumerate(w.solids):
        e = s.ext
        shape = (e[2], e[1], e[0])
        xo = np.fromfile(os.path.join(tmpdir, f"out{i}.bin"), dtype=np.float64).reshape((3,) + shape)
        lab = np.fromfile(os.path.join(tmpdir, f"lab{i}.bin"), dtype=np.int8).reshape(shape)
        dec = np.fromfile(os.path.join(tmpdir, f"dec{i}.bin"), dtype=np.int8).reshape(shape)
        raw = open(os.path.join(tmpdir, f"st{i}.bin"), "rb").read()
        outs.append((xo, lab, dec, raw))
    return st, outs
