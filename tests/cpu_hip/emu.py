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
           ("rmx_kernels.hip", "rmx_step.hip", "rmx_blur.hip", "rmx_plan.cpp",
            "rmx_core.cpp", "rmx_server.cpp")] + \
          [os.path.join(HERE, "hip_emu.cpp"), os.path.join(HERE, "run_case.cpp")]


def build(sanitize=True):
    srcs = SOURCES
    newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(HERE, "hip", "hip_runtime.h")]
                 + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")])
    if os.path.exists(EXE) and os.path.getmtime(EXE) > newest:
        return EXE
    flags = ["-std=c++20", "-g", "-O1", "-fno-omit-frame-pointer", "-Wno-unknown-attributes",
             "-Wno-unused-command-line-argument", "-I", HERE, "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-DRMX_EMU_REDZONES", "-ffp-contract=off"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = [CLANG] + flags + ["-x", "c++"] + srcs + ["-o", EXE + ".tmp", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(EXE + ".tmp", EXE)
    return EXE


def grid_line(w, n_solids):
    """The grid line of a case file: solids, n, h, origin, spacing, periodic."""
    sp = getattr(w, "spacing", (0.0, 0.0, 0.0))
    per = getattr(w, "periodic", (0, 0, 0))
    return (f"{n_solids} {w.grid_n[0]} {w.grid_n[1]} {w.grid_n[2]} {w.h!r} "
            f"{w.origin[0]!r} {w.origin[1]!r} {w.origin[2]!r} "
            + " ".join(repr(float(v)) for v in sp) + " "
            + " ".join(str(int(bool(v))) for v in per))


def run(w, tmpdir, r_s=2, r_max=4, normal_layers=2, precision=0, flags=0, reps=1,
        xi_normal=None, timeout=600, pre_flags=(), cus=None):
    """Write workload `w` to tmpdir, run the emulated library, return
    (status, [(xi_out, labels, decisions, stats_raw)])."""
    os.makedirs(tmpdir, exist_ok=True)
    lines = [grid_line(w, len(w.solids)),
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


def run_step(w, tmpdir, xi_n, labels_n, u, uf, dt, xi_next_init, xi_half_init, r_s=2, r_max=4,
             normal_layers=2, precision=0, flags=0, timeout=600):
    """One rmx_step call of the emulated library on workload `w` (boxes, shapes, layers;
    its xi is ignored).  Per solid: xi_n, labels_n, u, uf = (x, y, z faces), the initial
    xi_next and xi_half.  Returns (status, [(xi_next, labels_next, decisions, stats_raw,
    xi_half)])."""
    import types
    solids = []
    for i, s in enumerate(w.solids):
        solids.append(types.SimpleNamespace(lo=s.lo, ext=s.ext, n_layers=s.n_layers,
                                            shape=s.shape, xi=xi_next_init[i]))
    ww = types.SimpleNamespace(solids=solids, grid_n=w.grid_n, h=w.h, origin=w.origin,
                               spacing=getattr(w, "spacing", (0.0, 0.0, 0.0)),
                               periodic=getattr(w, "periodic", (0, 0, 0)))
    os.makedirs(tmpdir, exist_ok=True)
    with open(os.path.join(tmpdir, "step.txt"), "w") as f:
        f.write(f"{float(dt)!r}\n")
    for i in range(len(w.solids)):
        def put(name, a, dtype):
            np.ascontiguousarray(a, dtype=dtype).tofile(os.path.join(tmpdir, f"{name}{i}.bin"))
        put("xin", xi_n[i], np.float64)
        put("labn", labels_n[i], np.int8)
        put("u", u[i], np.float64)
        put("ufx", uf[i][0], np.float64)
        put("ufy", uf[i][1], np.float64)
        put("ufz", uf[i][2], np.float64)
        put("xhalf", xi_half_init[i], np.float64)
    try:
        st, outs = run(ww, tmpdir, r_s=r_s, r_max=r_max, normal_layers=normal_layers,
                       precision=precision, flags=flags, timeout=timeout)
    finally:
        os.remove(os.path.join(tmpdir, "step.txt"))
    res = []
    for i, (xo, lab, dec, raw) in enumerate(outs):
        half = np.fromfile(os.path.join(tmpdir, f"half{i}.bin"), dtype=np.float64).reshape(xo.shape)
        res.append((xo, lab, dec, raw, half))
    return st, res


def run_blur(w, tmpdir, xi, labels, eps, G, H_init, phi_init, tau_init, timeout=600):
    """rmx_blur then rmx_solid_stress of the emulated library on workload `w` (boxes,
    shapes, layers) with the given per-solid xi and labels.  Returns (status, H,
    [phi per solid], [tau per face orientation])."""
    import types
    solids = [types.SimpleNamespace(lo=s.lo, ext=s.ext, n_layers=s.n_layers, shape=s.shape,
                                    xi=xi[i]) for i, s in enumerate(w.solids)]
    ww = types.SimpleNamespace(solids=solids, grid_n=w.grid_n, h=w.h, origin=w.origin,
                               spacing=getattr(w, "spacing", (0.0, 0.0, 0.0)),
                               periodic=getattr(w, "periodic", (0, 0, 0)))
    os.makedirs(tmpdir, exist_ok=True)
    with open(os.path.join(tmpdir, "blur.txt"), "w") as f:
        f.write(f"{float(eps)!r} " + " ".join(repr(float(v)) for v in G) + "\n")
    put = lambda name, a, dt: np.ascontiguousarray(a, dtype=dt).tofile(
        os.path.join(tmpdir, name + ".bin"))
    for i in range(len(w.solids)):
        put(f"labin{i}", labels[i], np.int8)
        put(f"phiinit{i}", phi_init[i], np.float64)
    put("hinit", H_init, np.float64)
    for a in range(3):
        put(f"tauinit{a}", tau_init[a], np.float64)
    try:
        # the extrapolation runner's own outputs are not produced in this mode
        os.makedirs(tmpdir, exist_ok=True)
        for i, s in enumerate(solids):
            np.ascontiguousarray(s.xi, dtype=np.float64).tofile(os.path.join(tmpdir, f"xi{i}.bin"))
        lines = [grid_line(w, len(solids)), "2 4 2 0 0 1"]
        for s in solids:
            sh = s.shape
            vals = list(s.lo) + list(s.ext) + [s.n_layers, sh.kind]
            fl = list(map(float, sh.centre)) + list(map(float, sh.semi)) + \
                list(map(float, np.asarray(sh.rot).reshape(-1)))
            lines.append(" ".join(str(int(v)) for v in vals) + " " +
                         " ".join(repr(v) for v in fl) + " 0")
        with open(os.path.join(tmpdir, "case.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1")
        subprocess.run([build(), tmpdir], check=True, timeout=timeout, env=env)
    finally:
        os.remove(os.path.join(tmpdir, "blur.txt"))
    st = int(open(os.path.join(tmpdir, "status.txt")).read())
    get = lambda name, like: np.fromfile(os.path.join(tmpdir, name + ".bin"),
                                         dtype=np.float64).reshape(like.shape)
    H = get("hout", H_init)
    phis = [get(f"phiout{i}", phi_init[i]) for i in range(len(solids))]
    taus = [get(f"tauout{a}", tau_init[a]) for a in range(3)]
    return st, H, phis, taus


def read_h_without_phi(tmpdir, like):
    """H of the run_blur case's second rmx_blur call, made without phi outputs."""
    return np.fromfile(os.path.join(tmpdir, "hout_nophi.bin"), dtype=np.float64).reshape(
        like.shape)
