"""Tile choices saved by one process and loaded by another (helm_tiles_save /
helm_tiles_load): the second process skips the timing in its setup, and with the
same choices its solve is bit-identical to the first process's."""
import json
import os
import subprocess
import sys
import time

import numpy as np
import pytest
import torch

from tests.test_gpu_parity import H
from workloads import grf_velocity, load_iofd_table, point_source
from workloads.configs import omega_for_ppw

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PHYS, NPML = (36, 32, 44), 6   # a shape no other test uses, so this process times its tiles here

CHILD = r"""
import json, sys, time
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2608_22946_amd import helm
from workloads import grf_velocity, load_iofd_table, point_source
from workloads.configs import omega_for_ppw
phys, npml, h, path, out = json.loads(sys.argv[2]), int(sys.argv[3]), float(sys.argv[4]), sys.argv[5], sys.argv[6]
n = helm.tiles_load(path)
vel = grf_velocity(*phys, seed=51, corr_len=6.0)
omega = omega_for_ppw(float(vel.min()), h)
torch.zeros(1, device="cuda:0")
torch.cuda.synchronize()
t0 = time.perf_counter()
Hh = helm.Hierarchy(torch.from_numpy(vel), h, omega, npml, precision="fp32", table=load_iofd_table(), device="cuda:0")
torch.cuda.synchronize()
t = time.perf_counter() - t0
N = tuple(p + 2 * npml for p in phys)
f = torch.from_numpy(point_source(N, tuple(v // 2 for v in N), h)).to("cuda:0").to(torch.complex64)
u, its, rel, rc = Hh.solve(f, 1e-6)
np.save(out, u.cpu().numpy())
print(json.dumps({"loaded": n, "setup_s": t, "calls": int(its)}), flush=True)
"""


def test_tiles_saved_and_loaded_across_processes(tmp_path):
    from paper_2608_22946_amd import helm
    vel = grf_velocity(*PHYS, seed=51, corr_len=6.0)
    omega = omega_for_ppw(float(vel.min()), H)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Hh = helm.Hierarchy(torch.from_numpy(vel), H, omega, NPML, precision="fp32", table=load_iofd_table(),
                        device="cuda:0")
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t0
    N = tuple(p + 2 * NPML for p in PHYS)
    f = torch.from_numpy(point_source(N, tuple(v // 2 for v in N), H)).to("cuda:0").to(torch.complex64)
    u, its, rel, rc = Hh.solve(f, 1e-6)
    assert rc == 0
    path = tmp_path / "tiles.txt"
    helm.tiles_save(str(path))
    lines = path.read_text().splitlines()
    dims = [Hh.dims(l) for l in range(3)]
    mine = [ln for ln in lines[1:] if ln.split()[1] == "1" and
            tuple(int(v) for v in ln.split()[5:8]) in [tuple(d) for d in dims]]
    assert len(mine) == 6, lines   # three levels, two kernel families
    out = tmp_path / "u_child.npy"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(PHYS), str(NPML), str(H), str(path), str(out)],
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(f"\nsetup with timing {t_timed:.3f} s, with loaded choices {res['setup_s']:.3f} s; "
          f"{res['loaded']} entries loaded")
    assert res["loaded"] >= 6 and res["calls"] == int(its)
    assert res["setup_s"] < 0.5 * t_timed
    assert np.array_equal(np.load(out), u.cpu().numpy())
