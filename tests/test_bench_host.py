"""Host logic of bench.py without a GPU: its rotation-error helper agrees
with the oracle's, and the committed HBM-traffic record is used only while
every source it is keyed on is unchanged."""
import hashlib
import json
import os

import numpy as np

import bench
from oracle import lsgcpd_oracle as O


def _rot(axis, deg):
    axis = np.asarray(axis, dtype=np.float64)
    return O.se3_exp(np.concatenate([np.radians(deg) * axis / np.linalg.norm(axis),
                                     np.zeros(3)]))[:3, :3]


def test_rot_err_deg_matches_oracle():
    rng = np.random.default_rng(7)
    for deg in (0.0, 1e-7, 1e-3, 0.5, 30.0, 120.0, 179.0):
        G = _rot(rng.normal(size=3), rng.uniform(0, 180))
        R = G @ _rot(rng.normal(size=3), deg)
        got = bench.rot_err_deg(R, G)
        assert abs(got - deg) <= 1e-9 * max(1.0, deg)
        assert abs(got - O.rotation_error_deg(R, G)) <= 1e-9 * max(1.0, deg)


def test_traffic_record_keyed_on_its_sources(tmp_path):
    rec = json.load(open(os.path.join(bench.ROOT, "profiles",
                                      "estep_pairs_rgbd_20000x20000_traffic.json")))
    assert {s["path"] for s in rec["sources"]} == {
        "paper_2103_15039_amd/csrc/estep.hip", "paper_2103_15039_amd/csrc/api.hip",
        "paper_2103_15039_amd/csrc/order.hip"}
    for src in rec["sources"]:   # the record as it would be for today's sources
        src["sha256"] = hashlib.sha256(open(os.path.join(bench.ROOT, src["path"]),
                                            "rb").read()).hexdigest()
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(str(p)) == rec["bytes_per_launch"]
    rec["sources"][1]["sha256"] = "0" * 64     # one stale key: no figure
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(str(p)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.json")) is None
