"""Comparison of GPU results with the FP64 oracle.

First hits: every entry must be accepted by the oracle's tolerance-band rule
(bit equality wherever no slot of the entry has |margin| <= 1e-4 m).
Criticality: within 1e-6 absolute of the oracle's, where the oracle's value is
an interval [lo, hi] when trajectory pairs inside the band may flip.
"""
from __future__ import annotations

import numpy as np

import oracle

CRIT_TOL = 1e-6


def check(scene, gpu: dict, orc: "oracle.OracleResult", label: str = "", q: bool = True):
    H = scene.horizon
    k32 = gpu["first_hit"]
    assert k32 is not None and k32.shape == orc.k64.shape, label
    assert int(k32.min(initial=-1)) >= -1 and int(k32.max(initial=-1)) < H, f"{label}: first hit out of range"
    acc = oracle.accepted_first_hits(k32, orc)
    bad = np.flatnonzero(~acc)
    assert bad.size == 0, (f"{label}: {bad.size} first hits rejected, e.g. entry {bad[:5]} "
                           f"gpu {k32[bad[:5]]} oracle {orc.k64[bad[:5]]} strict {orc.kstrict[bad[:5]]}")
    for name, lo, hi, mid in (("object_crit", orc.obj_crit_lo, orc.obj_crit_hi, orc.obj_crit),
                              ("traj_crit", orc.traj_crit_lo, orc.traj_crit_hi, orc.traj_crit)):
        g = gpu[name]
        ok = (g >= lo - CRIT_TOL) & (g <= hi + CRIT_TOL)
        assert ok.all(), f"{label}: {name} outside oracle bounds, max dev {np.max(np.abs(g - mid))}"
    assert np.allclose(gpu["traj_prob"], orc.p, rtol=1e-14, atol=1e-17), f"{label}: traj_prob"
    if q and gpu.get("q") is not None and np.array_equal(orc.traj_crit_lo, orc.traj_crit_hi):
        assert np.allclose(gpu["q"], orc.q, rtol=0, atol=1e-12), f"{label}: q"
    if getattr(scene, "timeline", 0):
        check_timeline(scene, gpu, orc, label)
    exact = float(np.mean(k32 == orc.k64)) if k32.size else 1.0
    return exact


def check_timeline(scene, gpu: dict, orc: "oracle.OracleResult", label: str = ""):
    """Risk over time. The criticality per slot is monotone in the hit
    indicators, so it must lie in the oracle's interval from the latest and
    earliest first hits the band allows. The attribution moves by at most the
    probability mass of the combinations whose first hit the band leaves open.
    The GPU's own results must add up: the last slot and the attribution sum
    give the plain criticality."""
    for name, lo, hi, mid in (("crit_t", orc.obj_crit_t_lo, orc.obj_crit_t_hi, orc.obj_crit_t),
                              ("traj_crit_t", orc.traj_crit_t_lo, orc.traj_crit_t_hi, orc.traj_crit_t)):
        g = gpu[name]
        assert g is not None and g.shape == mid.shape, f"{label}: {name} shape"
        ok = (g >= lo - CRIT_TOL) & (g <= hi + CRIT_TOL)
        assert ok.all(), f"{label}: {name} outside oracle bounds, max dev {np.max(np.abs(g - mid))}"
    for name, mid, amb in (("attrib", orc.obj_attrib, orc.obj_amb_mass),
                           ("traj_attrib", orc.traj_attrib, orc.traj_amb_mass)):
        g = gpu[name]
        assert g is not None and g.shape == mid.shape, f"{label}: {name} shape"
        dev = np.abs(g - mid) - amb[:, None]
        assert np.all(dev <= CRIT_TOL), f"{label}: {name} off by {dev.max()} beyond the band's mass"
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
