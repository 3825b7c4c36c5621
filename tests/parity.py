"""Comparison of GPU results with the FP64 oracle.

First hits: every entry must be accepted by the oracle's tolerance-band rule
(bit equality wherever no slot of the entry has |margin| <= 1e-4 m).

Criticality (Sec. IV-D, IV-D.2): the oracle's risk step is recomputed from
the GPU's own first hits (an entry collides iff its accepted first hit is not
-1), so the comparison tests the reduction alone, on every scene whether or
not it has entries inside the band: q within 1e-12, traj_crit and
object_crit within 1e-6 absolute, and for time-resolved scenes the
criticality per slot and the attribution (the chronological scaling
recomputed from the GPU's first-hit slots) within 1e-6. As a second
assertion the criticality must also lie within 1e-6 of the oracle's interval
[value with every band pair counted as a miss, value with every band pair
counted as a hit]: criticality is monotone in the hit indicators.
"""
from __future__ import annotations

import numpy as np

import oracle

CRIT_TOL = 1e-6
Q_TOL = 1e-12

#: largest deviation seen by ``check`` since import, per output (reported by
#: the tests that want to print it)
max_dev: dict = {}


def _dev(name: str, got: np.ndarray, want: np.ndarray) -> float:
    d = float(np.max(np.abs(np.asarray(got, np.float64) - want))) if np.size(want) else 0.0
    max_dev[name] = max(max_dev.get(name, 0.0), d)
    return d


def check(scene, gpu: dict, orc: "oracle.OracleResult", label: str = "", q: bool = True):
    H = scene.horizon
    k32 = gpu["first_hit"]
    assert k32 is not None and k32.shape == orc.k64.shape, label
    assert int(k32.min(initial=-1)) >= -1 and int(k32.max(initial=-1)) < H, f"{label}: first hit out of range"
    acc = oracle.accepted_first_hits(k32, orc)
    bad = np.flatnonzero(~acc)
    assert bad.size == 0, (f"{label}: {bad.size} first hits rejected, e.g. entry {bad[:5]} "
                           f"gpu {k32[bad[:5]]} oracle {orc.k64[bad[:5]]} strict {orc.kstrict[bad[:5]]}")
    assert np.allclose(gpu["traj_prob"], orc.p, rtol=1e-14, atol=1e-17), f"{label}: traj_prob"
    model = int(getattr(scene, "risk", oracle.RISK_EXCLUSIVE))
    # the oracle's risk step on the GPU's accepted first hits
    q_r, tc_r, oc_r = oracle.risk_raw(orc.T, orc.pair_a, orc.pair_b, (k32 >= 0), orc.p, model)
    for name, want in (("object_crit", oc_r), ("traj_crit", tc_r)):
        d = _dev(name, gpu[name], want)
        assert d <= CRIT_TOL, f"{label}: {name} differs from the oracle's risk on the GPU's first hits by {d:.3e}"
    if q and gpu.get("q") is not None:
        d = _dev("q", gpu["q"], q_r)
        assert d <= Q_TOL, f"{label}: q differs from the oracle's risk on the GPU's first hits by {d:.3e}"
    # second assertion: inside the interval the band allows
    for name, lo, hi in (("object_crit", orc.obj_crit_lo, orc.obj_crit_hi),
                         ("traj_crit", orc.traj_crit_lo, orc.traj_crit_hi)):
        g = gpu[name]
        ok = (g >= lo - CRIT_TOL) & (g <= hi + CRIT_TOL)
        assert ok.all(), f"{label}: {name} outside the oracle's band interval"
    if getattr(scene, "timeline", 0):
        check_timeline(scene, gpu, orc, label)
    exact = float(np.mean(k32 == orc.k64)) if k32.size else 1.0
    return exact


def check_timeline(scene, gpu: dict, orc: "oracle.OracleResult", label: str = ""):
    """Risk over time: the oracle's chronological scaling recomputed from the
    GPU's first-hit slots; then, as second assertions, the criticality per
    slot inside the oracle's interval from the latest and earliest first hits
    the band allows, and the GPU's own results adding up (the last slot and
    the attribution sum give the plain criticality)."""
    k32 = np.asarray(gpu["first_hit"]).astype(np.int32)
    model = int(getattr(scene, "risk", oracle.RISK_EXCLUSIVE))
    tct, oct_, tat, oat = oracle.risk_timeline_raw(orc.T, int(scene.horizon), orc.pair_a, orc.pair_b, k32,
                                                   orc.p, model)
    for name, want in (("crit_t", oct_), ("traj_crit_t", tct), ("attrib", oat), ("traj_attrib", tat)):
        g = gpu[name]
        assert g is not None and g.shape == want.shape, f"{label}: {name} shape"
        d = _dev(name, g, want)
        assert d <= CRIT_TOL, f"{label}: {name} differs from the oracle's scaling on the GPU's first hits by {d:.3e}"
    for name, lo, hi in (("crit_t", orc.obj_crit_t_lo, orc.obj_crit_t_hi),
                         ("traj_crit_t", orc.traj_crit_t_lo, orc.traj_crit_t_hi)):
        g = gpu[name]
        ok = (g >= lo - CRIT_TOL) & (g <= hi + CRIT_TOL)
        assert ok.all(), f"{label}: {name} outside the oracle's band interval"
    assert np.allclose(gpu["crit_t"][:, -1], gpu["object_crit"], rtol=0, atol=1e-12), f"{label}: crit_t end"
    assert np.allclose(gpu["attrib"].sum(axis=1), gpu["object_crit"], rtol=0, atol=1e-12), f"{label}: attrib sum"
    assert np.allclose(gpu["traj_crit_t"][:, -1], gpu["traj_crit"], rtol=0, atol=1e-12), f"{label}: traj_crit_t end"
    assert np.all(np.diff(gpu["traj_crit_t"], axis=1) >= -1e-12), f"{label}: criticality decreases over time"


def same_results(a: dict, b: dict, label: str = ""):
    """Bit equality of first hits and criticality between two GPU paths."""
    for k in ("first_hit", "object_crit", "traj_crit", "traj_prob", "q",
              "crit_t", "traj_crit_t", "attrib", "traj_attrib"):
        if a.get(k) is None or b.get(k) is None:
            continue
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.shape == y.shape and np.array_equal(x, y), f"{label}: {k} differs"
