"""The serving loop on the GPU: HBM-budgeted admission, resident fields, batching of
requests from several simulations (different grids, layer counts and precisions) across
streams.  Each served result must equal, bit for bit, the result of the same input
extrapolated alone through a context (the per-cell arithmetic does not depend on the
batch), and match the oracle within the stated tolerance."""
import numpy as np
import pytest

from paper_2104_00095_amd import synth
from tests.helpers import rel_err, run_oracle

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
GiB = 1 << 30


def _sims():
    """Six small simulations: grids 32..64, 1-5 ellipsoids, L 4-6, FP64 / FP32-accumulate."""
    out = []
    for i, (n, k, L) in enumerate([(32, 2, 4), (48, 3, 5), (64, 5, 4), (40, 1, 6), (56, 4, 5),
                                   (32, 3, 6)]):
        w = synth.suspension(seed=100 + i, n_solids=k, grid_n=(n, n, n), h=1.0 / n,
                             n_layers=L, semi_lo=0.08, semi_hi=0.16)
        out.append((w, i % 2))
    return out


def _template(w):
    from paper_2104_00095_amd import rmx
    return [rmx.solid_template(s.lo, s.ext, rmx.shape(s.shape.kind, s.shape.centre,
                                                      s.shape.semi, s.shape.rot), s.n_layers)
            for s in w.solids]


def _solo(ctx, w, precision):
    """Each solid extrapolated alone through a context, on its own copy of the input."""
    import torch
    from paper_2104_00095_amd import fields, rmx
    dw = fields.upload(w)
    st, stats = ctx.extrapolate(dw.grid, dw.solids, rmx.options(precision=precision,
                                                                flags=rmx.FLAG_PER_SOLID),
                                check=False)
    torch.cuda.synchronize()
    return [(dw.xi[i].cpu().numpy(), dw.labels[i].cpu().numpy()) for i in range(len(w.solids))]


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_00095_amd import rmx
    c = rmx.Context(0)
    yield c
    c.close()


def test_served_equals_solo_and_oracle(ctx):
    from paper_2104_00095_amd import rmx
    sims = _sims()
    srv = rmx.Server(0, 8 * GiB, 3)
    try:
        ids = []
        for w, prec in sims:
            sid = srv.register(rmx.grid(w.grid_n, w.h, w.origin), _template(w))
            for j, s in enumerate(w.solids):
                srv.upload(sid, j, s.xi)
            ids.append(sid)
        # two rounds, submitted in different orders, so that batches differ
        for order in (list(range(len(sims))), list(reversed(range(len(sims))))):
            for i in order:
                for j, s in enumerate(sims[i][0].solids):
                    srv.upload(ids[i], j, s.xi)
            tickets = {i: srv.submit(ids[i], rmx.options(precision=sims[i][1])) for i in order}
            for i in order:
                w, prec = sims[i]
                st, lat, stats = srv.wait(tickets[i], len(w.solids))
                assert st == 0, (i, st)
                assert lat > 0.0
                solo = _solo(ctx, w, prec)
                for j, s in enumerate(w.solids):
                    xi, lab = srv.download(ids[i], j, s.ext)
                    assert np.array_equal(lab, solo[j][1]), (i, j)
                    assert np.array_equal(xi.view(np.uint64), solo[j][0].view(np.uint64)), (i, j)
                    ost, xo, lo, do, so = run_oracle(w, s)
                    assert np.array_equal(lab, lo)
                    assert stats[j]["n_band"][1:17] == [int(v) for v in so[1:17]]
                    assert rel_err(xi, xo, lo > 0) <= TOL[prec], (i, j)
        used, peak = srv.usage()
        assert 0 < used <= peak <= 8 * GiB
        for sid in ids:
            srv.release(sid)
    finally:
        srv.close()


def test_budget_admission_and_errors():
    from paper_2104_00095_amd import rmx
    w = synth.suspension(seed=7, n_solids=3, grid_n=(48, 48, 48), h=1.0 / 48, n_layers=4,
                         semi_lo=0.08, semi_hi=0.14)
    fields_bytes = sum(((24 * int(np.prod(s.ext)) + 255) // 256 + (int(np.prod(s.ext)) + 255)
                        // 256) * 256 for s in w.solids)
    g = rmx.grid(w.grid_n, w.h, w.origin)
    # fields alone exceed the budget
    srv = rmx.Server(0, fields_bytes // 2, 2)
    try:
        with pytest.raises(rmx.RmxError) as ei:
            srv.register(g, _template(w))
        assert ei.value.status == rmx.E_BUDGET
    finally:
        srv.close()
    # a budget that holds the fields of two copies plus about one call's workspace:
    # the requests are admitted one lane at a time and all complete
    ws = rmx.workspace_size(g, _template(w))
    srv = rmx.Server(0, 2 * fields_bytes + ws + ws // 2, 3)
    try:
        a = srv.register(g, _template(w))
        b = srv.register(g, _template(w))
        for sid in (a, b):
            for j, s in enumerate(w.solids):
                srv.upload(sid, j, s.xi)
        ta, tb = srv.submit(a), srv.submit(b)
        assert srv.wait(ta, len(w.solids))[0] == 0
        assert srv.wait(tb, len(w.solids))[0] == 0
        used, peak = srv.usage()
        assert peak <= 2 * fields_bytes + ws + ws // 2
        xa, la = srv.download(a, 0, w.solids[0].ext)
        xb, lb = srv.download(b, 0, w.solids[0].ext)
        assert np.array_equal(la, lb) and np.array_equal(xa.view(np.uint64), xb.view(np.uint64))
        # bad requests
        with pytest.raises(rmx.RmxError) as ei:
            srv.submit(987654)
        assert ei.value.status == rmx.E_NOTFOUND
        assert srv.wait(123456789)[0] == rmx.E_NOTFOUND
        with pytest.raises(rmx.RmxError) as ei:
            srv.submit(a, rmx.options(r_s=0))
        assert ei.value.status == rmx.E_ARG
        srv.release(a)
        with pytest.raises(rmx.RmxError) as ei:
            srv.release(a)
        assert ei.value.status == rmx.E_NOTFOUND
    finally:
        srv.close()
