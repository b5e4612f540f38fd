"""The FP32 noise floor of the seeded-body scene (tests/golden/fp32_floor.json,
written by tests/golden/fp32_floor.py with the oracle alone): every float32
input moved by one ulp changes the FP64 render by this much.  This test
recomputes the stored worst pixels, so the fixture is reproducible from
committed code, and checks what the numbers are used for: the floor is set
by the rays (the camera and the sample positions), not by the field's
parameters, and it grows with the density gain inside the body."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location("fp32_floor", os.path.join(HERE, "golden", "fp32_floor.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_fixture_reproduces_and_orders_the_sources():
    fx = json.load(open(os.path.join(HERE, "golden", "fp32_floor.json")))
    f100, f300 = fx["sigma_inside"]["100"], fx["sigma_inside"]["300"]
    # the worst pixels of the ray-driven groups, recomputed
    mod = _script()
    pid = np.array([f100["camera"]["worst"][0][0], f100["all"]["worst"][0][0]])
    got = mod.floor_at(100.0, pid, groups=("camera", "all"))
    assert abs(got["camera"][0] - f100["camera"]["worst"][0][1]) <= 1e-12
    assert abs(got["all"][1] - f100["all"]["worst"][0][1]) <= 1e-12
    # the field's parameters alone stay far below the FP32 path's 1e-5 bound;
    # rounding the camera (as the kernels' float32 ray set-up does) does not
    for f in (f100, f300):
        assert f["field"]["max"] < 1e-6
        assert f["camera"]["max"] > f["pose"]["max"] > f["field"]["max"]
    # a larger density gain sharpens the body's edge and raises every row
    for g in ("field", "pose", "camera", "all"):
        assert f300[g]["max"] > f100[g]["max"]
