"""Device-side evaluation (torch, FP64) of the affine+sine reference-map fields of
``synth``, for workloads too large to build on the host: the same formula,
xi(x) = c + A (x - c) + amp * sum_m u_m sin(2 pi k_m . x + theta_m + phase).  Input
generation only: none of the extrapolation method's arithmetic is here.
"""
import math


def affine_sine_field(spec, h, origin=(0.0, 0.0, 0.0), phase_shift=0.0, device="cuda:0"):
    """float64 [3, ext2, ext1, ext0] on `device` for a ``synth.SolidSpec``."""
    import torch
    f64 = torch.float64
    lo, ext = spec.lo, spec.ext
    x = (origin[0] + (torch.arange(lo[0], lo[0] + ext[0], dtype=f64, device=device) + 0.5) * h
         ).view(1, 1, -1)
    y = (origin[1] + (torch.arange(lo[1], lo[1] + ext[1], dtype=f64, device=device) + 0.5) * h
         ).view(1, -1, 1)
    z = (origin[2] + (torch.arange(lo[2], lo[2] + ext[2], dtype=f64, device=device) + 0.5) * h
         ).view(-1, 1, 1)
    c, A = spec.c, spec.A
    X = (x - float(c[0]), y - float(c[1]), z - float(c[2]))
    xi = torch.empty((3, ext[2], ext[1], ext[0]), dtype=f64, device=device)
    for a in range(3):
        xi[a] = float(c[a]) + (float(A[a, 0]) * X[0] + float(A[a, 1]) * X[1] +
                               float(A[a, 2]) * X[2])
    if spec.amp != 0.0:
        us, ks, ths = spec.modes
        for u, k, th in zip(us, ks, ths):
            s = torch.sin(2.0 * math.pi * (float(k[0]) * x + float(k[1]) * y + float(k[2]) * z)
                          + (float(th) + phase_shift))
            for a in range(3):
                xi[a] += (spec.amp * float(u[a])) * s
    return xi
