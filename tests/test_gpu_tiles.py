"""Tile choices saved by one process and loaded by another (helm_tiles_save /
helm_tiles_load): the second process skips the timing in its setup (its setup of the
loaded shape takes well under that of a fresh shape of about the same size, both after
a warm-up setup with fixed tiles), and with the same choices its solve is
bit-identical to the first process's."""
import json
import os
import subprocess
import sys

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
table = load_iofd_table()
def setup(ph, **kw):
    v = grf_velocity(*ph, seed=51, corr_len=6.0)
    om = omega_for_ppw(float(v.min()), h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Hx = helm.Hierarchy(torch.from_numpy(v), h, om, npml, precision="fp32", table=table, device="cuda:0", **kw)
    torch.cuda.synchronize()
    return Hx, time.perf_counter() - t0
setup((12, 12, 12), tile_tz=4, tile_split=0)          # warm-up: loads the kernels, times nothing
_, t_fresh = setup((phys[0] + 4, phys[1], phys[2]))   # a shape of about the same size, timed here
Hh, t = setup(phys)                                   # the loaded shape
N = tuple(p + 2 * npml for p in phys)
f = torch.from_numpy(point_source(N, tuple(v // 2 for v in N), h)).to("cuda:0").to(torch.complex64)
u, its, rel, rc = Hh.solve(f, 1e-6)
np.save(out, u.cpu().numpy())
print(json.dumps({"loaded": n, "setup_s": t, "setup_fresh_s": t_fresh, "calls": int(its)}), flush=True)
"""


def test_tiles_saved_and_loaded_across_processes(tmp_path):
    from paper_2608_22946_amd import helm
    vel = grf_velocity(*PHYS, seed=51, corr_len=6.0)
    omega = omega_for_ppw(float(vel.min()), H)
    Hh = helm.Hierarchy(torch.from_numpy(vel), H, omega, NPML, precision="fp32", table=load_iofd_table(),
                        device="cuda:0")
    N = tuple(p + 2 * NPML for p in PHYS)
    f = torch.from_numpy(point_source(N, tuple(v // 2 for v in N), H)).to("cuda:0").to(torch.complex64)
    u, its, rel, rc = Hh.solve(f, 1e-6)
    assert rc == 0
    path = tmp_path / "tiles.txt"
    helm.tiles_save(str(path))
    lines = path.read_text().splitlines()
    dims = [Hh.dims(l) for l in range(3)]
    mine = [ln for ln in lines[1:] if ln.split()[1] == "1" and ln.split()[5] == "1" and
            tuple(int(v) for v in ln.split()[6:9]) in [tuple(d) for d in dims]]
    assert len(mine) == 6, lines   # three levels, two kernel families
    out = tmp_path / "u_child.npy"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(PHYS), str(NPML), str(H), str(path), str(out)],
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(f"\nsecond process: setup of a fresh shape {res['setup_fresh_s']:.4f} s, of the loaded shape "
          f"{res['setup_s']:.4f} s; {res['loaded']} entries loaded")
    assert res["loaded"] >= 6 and res["calls"] == int(its)
    assert res["setup_s"] < 0.5 * res["setup_fresh_s"]
    assert np.array_equal(np.load(out), u.cpu().numpy())
    # choices recorded for another GPU architecture are read but not used
    arch = lines[1].split()[0]
    foreign = tmp_path / "foreign.txt"
    foreign.write_text(lines[0] + "\n" + " ".join(["gfx_other"] + lines[1].split()[1:]) + "\n")
    assert arch != "gfx_other" and helm.tiles_load(str(foreign)) == 0
