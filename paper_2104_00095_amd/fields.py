"""Move synthetic workloads into device memory and describe them to the library.

Marshalling only: host numpy fields are copied into torch tensors on the GPU, and one
``rmx.Solid`` descriptor is built per solid.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import rmx


@dataclass
class DeviceWorkload:
    grid: rmx.Grid
    solids: List[rmx.Solid]
    xi: list
    labels: list
    decisions: list
    xi_in: list = field(default_factory=list)   # pristine copies for resets

    def array(self):
        return (rmx.Solid * len(self.solids))(*self.solids)

    def reset(self):
        """Restore the input fields (the call writes band cells in place)."""
        for a, b in zip(self.xi, self.xi_in):
            a.copy_(b)


def upload(w, device="cuda:0", decisions=False, keep_input=True, xi_normal=None):
    import torch
    g = rmx.grid(w.grid_n, w.h, w.origin, spacing=getattr(w, "spacing", None),
                 periodic=getattr(w, "periodic", None))
    solids, xis, labs, decs, ins = [], [], [], [], []
    for idx, s in enumerate(w.solids):
        xi = torch.from_numpy(np.ascontiguousarray(s.xi)).to(device)
        lab = torch.empty((s.ext[2], s.ext[1], s.ext[0]), dtype=torch.int8, device=device)
        dec = torch.empty_like(lab) if decisions else None
        xn = None
        if xi_normal is not None and xi_normal[idx] is not None:
            xn = torch.from_numpy(np.ascontiguousarray(xi_normal[idx])).to(device)
        shp = rmx.shape(s.shape.kind, s.shape.centre, s.shape.semi, s.shape.rot)
        solids.append(rmx.solid(s.lo, s.ext, shp, s.n_layers, xi, lab, xi_normal=xn,
                                decisions=dec))
        xis.append(xi)
        labs.append(lab)
        decs.append(dec)
        if keep_input:
            ins.append(xi.clone())
    return DeviceWorkload(g, solids, xis, labs, decs, ins)
