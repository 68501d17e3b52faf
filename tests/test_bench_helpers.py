"""Host-side helpers of bench.py (no GPU): kernel naming, the serving
sample's caps, and the extra DD-cycle lines of the default run driven
through a stand-in library (so the JSON contract is exercised on the CPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_kernel_name_follows_layout_and_threads():
    import bench
    assert bench.kernel_name(3, 256) == "sweep_patch_kernel"
    assert bench.kernel_name(2, 256) == "sweep_patch1_kernel"
    assert bench.kernel_name(1, 64) == "sweep_node_kernel"
    assert bench.kernel_name(4, 512) == "sweep_stream_kernel"
    # several workgroups per subdomain (threads per subdomain above 1024)
    assert bench.kernel_name(4, 2048) == "sweep_stream_coop_kernel"


def test_serve_sample_keeps_stream_order_and_caps():
    import bench
    import workloads
    wls = workloads.c5(n_requests=400)
    got = bench.serve_sample(wls, 30, 40000, 2500)
    assert 0 < len(got) <= 30
    pos = [wls.index(w) for w in got]
    assert pos == sorted(pos)
    for w in got:
        assert (w.nx * w.P + 1) * (w.ny * w.P + 1) <= 40000
        assert ((w.nx // w.sx) * w.P + 1) * ((w.ny // w.sy) * w.P + 1) <= 2500
    # every skipped request before the last kept one breaks a cap
    kept = set(pos)
    for i in range(pos[-1]):
        if i not in kept:
            w = wls[i]
            assert ((w.nx * w.P + 1) * (w.ny * w.P + 1) > 40000
                    or ((w.nx // w.sx) * w.P + 1) * ((w.ny // w.sy) * w.P + 1) > 2500)


_STUB = r'''
import sys, types, argparse, json
import numpy as np
sys.path.insert(0, ROOT)
import torch
real_randn, real_gen = torch.randn, torch.Generator
torch.randn = lambda *a, **k: real_randn(*a, dtype=k.get("dtype", torch.float64))
torch.Generator = lambda device=None: real_gen()
class Ev:
    def __init__(self, **k): pass
    def record(self, s=None): pass
    def elapsed_time(self, o): return 5.0
torch.cuda.Event = Ev
torch.cuda.Stream = lambda: object()
torch.cuda.synchronize = lambda: None
torch.cuda.set_device = lambda d: None
W = types.ModuleType("paper_2606_21695_amd.wavedd")
W.DD_FP64, W.DD_FP32 = 0, 1
W.require_gpu = lambda: None
class Prob:
    def __init__(self, wl, **k): self.h = "h"
    def close(self): pass
W.Problem = Prob
W.dd_sizes = lambda h: {"n_iface": 10, "n_global": 100}
W.dd_set_state = lambda h, g: None
W.dd_time_sweep = lambda h, steps, it: (20.0, 1.6e9)
W.dd_apply_operator_device = lambda h, x, y, s: None
W.dd_layout = lambda h: (4, 2048)
W.dd3_mesh_coords = lambda *a: (np.zeros(8), np.zeros(8), np.zeros(8))
W.dd_default_options = lambda **k: k
W.dd3_setup = lambda *a, **k: "h3"
W.dd3_sizes = lambda h: {"n_iface": 10, "n_global": 100, "n_sub": 8, "n_local": 343}
W.dd3_sweep = lambda *a, **k: None
W.dd3_time_sweep = lambda h, steps, it: (5.0, 1.5e9)
W.dd3_apply_operator_device = lambda h, x, y, s: None
W.dd3_time_steps = lambda h: np.array([28])
W.dd3_destroy = lambda h: None
pkg = types.ModuleType("paper_2606_21695_amd")
pkg.wavedd = W
sys.modules["paper_2606_21695_amd"] = pkg
sys.modules["paper_2606_21695_amd.wavedd"] = W
import bench
a = argparse.Namespace(config="c2", precision="fp64", steps=5, layout="auto", no_cpu=False,
                       box_solve=False, protocol=False, warmup=1)
print(json.dumps(bench.other_workloads(a)))
'''


def test_other_workloads_lines_through_a_stand_in_library():
    code = "ROOT = %r\n" % ROOT + _STUB
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    c3, c6 = out["c3_protocol_fp64"], out["c6_protocol_fp64"]
    assert "error" not in c3 and "error" not in c6, out
    assert "error" not in out["c3_protocol_fp32"], out
    assert out["c3_protocol_fp32"]["roofline"]["byte_per_dof_update"] == 40
    assert c3["value"] == pytest.approx(1.6e9 / 20e-3)
    assert c3["config"]["kernel"] == "sweep_stream_coop_kernel"
    assert c3["roofline"]["bound"] == "hbm" and c3["roofline"]["unit"] == "GB/s"
    assert c3["roofline"]["achieved"] == pytest.approx(80 * 1.6e9 / 20e-3 / 1e9)
    assert c6["value"] == pytest.approx(1.5e9 / 5e-3)
    assert c6["roofline"]["bound"] == "alu" and c6["roofline"]["peak"] == 78.6
    # the stand-in events report 5 ms over 50 operator evaluations
    assert c6["dd_cycle_over_operator"] == pytest.approx(5.0 / (5.0 / 50))
    assert c3["dd_cycle_over_operator"] == pytest.approx(20.0 / (5.0 / 50))
