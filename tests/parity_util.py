"""Helpers for the GPU-vs-oracle parity tests (not collected by pytest)."""
from __future__ import annotations

import numpy as np

DEAD = np.uint64(0xFFFFFFFFFFFFFFFF)
PHOTON = 2


def oracle_stores(orc, init, caps):
    st = [orc.Store(caps[0]), orc.Store(caps[1]), orc.Store(caps[2], with_events=False)]
    for s, cols in zip(st, init):
        s.load(cols)
    return st


def oracle_field(orc, w, grids=None):
    from paper_1412_6426_amd import workloads as W
    f = w.field
    if f.kind == W.FIELD_YEE:
        return orc.Field(kind=orc.FIELD_YEE, grid=grids, dx=f.grid_dx, origin=f.grid_origin)
    return orc.Field(kind=f.kind, e0=f.e0, b0=f.b0, amp=f.amp, omega=f.omega, phase=f.phase)


def oracle_params(orc, w, **over):
    kw = dict(dt=w.dt, eps_r=w.eps_r, kappa=w.kappa, t0=w.t0, adaptive=w.adaptive,
              emission=w.emission, pairs=w.pairs, push_photons=w.push_photons, seed=w.seed)
    kw.update(over)
    return orc.Params(**kw)


def _sorted(c):
    order = np.lexsort((c["birth"], c["parent"], c["id"]))
    return {k: (v[order] if v is not None else None) for k, v in c.items()}


def compare_species(gpu, orc_cols, species, rtol=1e-12, label="", wtol=0.0, floor=(1.0, 1.0)):
    """Bit-exact ids, parents, births (and event counts for leptons); momenta and positions
    within rtol of max(|v|, floor) (floor: momentum and position scales, 1 by default);
    weights exact, or within wtol relative where thinning has rescaled them (its factor is
    a ratio of sums taken in different orders on the two sides).  Removed photons are
    compared by count."""
    g = dict(gpu)
    o = dict(orc_cols)
    if species == PHOTON:
        gd, od = g["id"] == DEAD, o["id"] == DEAD
        assert int(gd.sum()) == int(od.sum()), f"{label}: removed photons differ"
        g = {k: v[~gd] for k, v in g.items()}
        o = {k: (v[~od] if v is not None else None) for k, v in o.items()}
    assert len(g["id"]) == len(o["id"]), f"{label}: count {len(g['id'])} vs {len(o['id'])}"
    g, o = _sorted(g), _sorted(o)
    assert np.array_equal(g["id"], o["id"]), f"{label}: ids differ"
    assert np.array_equal(g["parent"], o["parent"]), f"{label}: parents differ"
    assert np.array_equal(g["birth"], o["birth"]), f"{label}: births differ"
    if species != PHOTON and o.get("n_events") is not None:
        assert np.array_equal(g["n_events"], o["n_events"]), f"{label}: event counts differ"
    if wtol == 0.0:
        assert np.array_equal(g["w"], o["w"]), f"{label}: weights differ"
    else:
        np.testing.assert_allclose(g["w"], o["w"], rtol=wtol, atol=0, err_msg=label)
    worst = {}
    for grp, fl in ((("px", "py", "pz"), floor[0]), (("x", "y", "z"), floor[1])):
        a = np.stack([g[c] for c in grp], 1)
        b = np.stack([o[c] for c in grp], 1)
        scale = np.maximum(np.linalg.norm(b, axis=1), fl)
        err = (np.abs(a - b).max(1) / scale) if len(a) else np.zeros(0)
        worst[grp[0]] = float(err.max()) if len(err) else 0.0
        assert worst[grp[0]] <= rtol, f"{label}: {grp} rel err {worst[grp[0]]:.3e}"
    return worst


def compare_all(engine, ostores, inst=0, rtol=1e-12, label="", wtol=0.0, floor=(1.0, 1.0)):
    out = {}
    for s in range(3):
        out[s] = compare_species(engine.read(inst, s), ostores[s].view(), s, rtol,
                                 f"{label} species {s}", wtol=wtol, floor=floor)
    return out
