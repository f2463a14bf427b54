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


def compare_species(gpu, orc_cols, species, rtol=1e-12, label="", wtol=0.0,
                    pos_floor=1.0, p_scale=None):
    """Bit-exact ids, parents, births (and event counts for leptons); momenta within rtol of
    each particle's own |p| (oracle side; a particle at rest must match exactly), or of
    p_scale(oracle columns, sorted) where a test derives a larger per-particle scale;
    positions within rtol of max(|x|, pos_floor); weights exact, or within wtol relative where
    thinning has rescaled them (its factor is a ratio of sums taken in different orders on the
    two sides).  Removed photons are compared by count."""
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
    for grp in (("px", "py", "pz"), ("x", "y", "z")):
        a = np.stack([g[c] for c in grp], 1)
        b = np.stack([o[c] for c in grp], 1)
        if grp[0] == "px":
            scale = np.linalg.norm(b, axis=1) if p_scale is None else p_scale(o)
        else:
            scale = np.maximum(np.linalg.norm(b, axis=1), pos_floor)
        d = np.abs(a - b).max(1) if len(a) else np.zeros(0)
        exact = scale == 0.0
        assert np.all(d[exact] == 0.0), f"{label}: {grp} differ where the oracle's is 0"
        err = d[~exact] / scale[~exact]
        worst[grp[0]] = float(err.max()) if len(err) else 0.0
        assert worst[grp[0]] <= rtol, f"{label}: {grp} rel err {worst[grp[0]]:.3e}"
    return worst


def lepton_birth_momentum(photons):
    """A lepton's momentum at its birth in a pure magnetic field, from the stores: Boris
    keeps |p| there and an emission takes |k| off |p| (k along p), so |p| at birth is the
    lepton's |p| plus the |k| of every photon it emitted (photons are found by their parent
    id; the removed ones keep k and parent in their slots)."""
    kabs = np.sqrt(photons["px"] ** 2 + photons["py"] ** 2 + photons["pz"] ** 2)
    ids, inv = np.unique(photons["parent"], return_inverse=True)
    emitted = np.bincount(inv, weights=kabs)

    def scale(o):
        pabs = np.sqrt(o["px"] ** 2 + o["py"] ** 2 + o["pz"] ** 2)
        at = np.minimum(np.searchsorted(ids, o["id"]), len(ids) - 1)
        mine = ids[at] == o["id"] if len(ids) else np.zeros(len(pabs), bool)
        return pabs + np.where(mine, emitted[at] if len(ids) else 0.0, 0.0)
    return scale


def compare_all(engine, ostores, inst=0, rtol=1e-12, label="", wtol=0.0, pos_floor=1.0,
                p_scale=None):
    out = {}
    for s in range(3):
        out[s] = compare_species(engine.read(inst, s), ostores[s].view(), s, rtol,
                                 f"{label} species {s}", wtol=wtol, pos_floor=pos_floor,
                                 p_scale=None if p_scale is None else p_scale[s])
    return out


# Fields of the per-step record that both sides keep (the GPU's record also holds the step
# index and how its kernels spread the work: wavefront iterations and early decisions).
EXACT_COUNTS = ("n_start", "advanced", "emitted", "pairs", "dropped", "saturated",
                "near_threshold", "nsub_near_int", "nsub_clamped", "nonfinite", "substeps",
                "nsub_refined", "children_advanced", "deferred", "nsub_hist", "photon_hist")
STATUS_BITS = (("dropped", 1), ("nonfinite", 2), ("saturated", 4), ("nsub_clamped", 8))


def compare_stats(gpu_steps, orc_steps, label="", probabilities=True, float_rtol=None):
    """Every field of the GPU's per-step record against the oracle's record of the same step:
    the counters and both histograms exactly; the radiated energy within (n + 2) 2^-53
    relative, n the step's emissions (the bound for sums of n positive terms taken in any
    order, at least 1e-12); the largest emission and pair probabilities within 1e-12 relative
    (probabilities=False skips them, for the FP32 rates of the mixed form; float_rtol, where
    a test has measured the problem's own conditioning, replaces both tolerances); the status
    bits as the oracle's counters set them; and on the GPU side alone, at most as many
    low-occupancy wavefront iterations as iterations."""
    assert len(gpu_steps) == len(orc_steps), f"{label}: {len(gpu_steps)} vs {len(orc_steps)} steps"
    for n, (g, o) in enumerate(zip(gpu_steps, orc_steps)):
        where = f"{label}: step {n}"
        for f in EXACT_COUNTS:
            assert list(np.atleast_1d(g[f])) == list(np.atleast_1d(o[f])), \
                f"{where}: {f} {g[f]} vs {o[f]}"
        tol = max(1e-12, (g["emitted"] + 2) * 2.0 ** -53)
        ptol = 1e-12
        if float_rtol is not None:
            tol = ptol = float_rtol
        assert abs(g["photon_energy"] - o["photon_energy"]) <= tol * abs(o["photon_energy"]), \
            f"{where}: photon_energy {g['photon_energy']!r} vs {o['photon_energy']!r}"
        if probabilities:
            for f in ("max_p_emit", "max_p_pair"):
                assert abs(g[f] - o[f]) <= ptol * abs(o[f]), f"{where}: {f} {g[f]!r} vs {o[f]!r}"
        bits = sum(b for f, b in STATUS_BITS if o[f] > 0)
        assert g["status"] == bits, f"{where}: status {g['status']} vs {bits}"
        assert 0 <= g["low_occupancy_iters"] <= g["wave_iters"], where


def merge_stats(per_instance):
    """The oracle's records of separate single-instance runs added up step by step, as one
    batched GPU step records them: counters and histograms summed, the largest probabilities
    maximised (an instance that stopped early contributes nothing after its last step)."""
    K = max(len(r) for r in per_instance)
    out = []
    for n in range(K):
        rows = [r[n] for r in per_instance if n < len(r)]
        m = {}
        for f in rows[0]:
            if f in ("max_p_emit", "max_p_pair"):
                m[f] = max(r[f] for r in rows)
            elif isinstance(rows[0][f], list):
                m[f] = [sum(v) for v in zip(*(r[f] for r in rows))]
            else:
                m[f] = sum(r[f] for r in rows)
        out.append(m)
    return out
