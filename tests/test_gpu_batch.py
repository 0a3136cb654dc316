"""GPU parity of batched right-hand sides (helm_options.batch): several sources
advanced together through one set of launches, each in its own slot.

Every right-hand side of a batched solve is compared with the FP64 oracle's
solution (tol 1e-10) at the converged-solution bar (1e-5; reading of the FP32
tolerance in the parity module), and with the same right-hand side solved
alone on the GPU: slots share launches but not arithmetic, so with the tiling
fixed the results, preconditioner counts and residuals are bit-identical.
"""
import numpy as np
import pytest
import torch

from tests.test_gpu_parity import H, rel, to_np
from workloads import grf_velocity, load_iofd_table, point_source
from workloads.configs import omega_for_ppw

pytestmark = pytest.mark.gpu

N_PHYS, NPML = 44, 10
N = N_PHYS + 2 * NPML
# sources at different depths (one close to the PML) so that the slots need different numbers of
# preconditioner calls and leave the batch at different times; one zero right-hand side
SOURCES = [(N // 2, N // 2, N // 2), (NPML + 3, N // 2 + 5, N // 2 - 4), (N // 2 - 7, NPML + 4, N // 2 + 6),
           None, (N // 2 + 9, N // 2 - 8, NPML + 2)]


def _sources(dtype):
    out = []
    for sp in SOURCES:
        out.append(np.zeros((N + 1,) * 3, dtype) if sp is None else point_source((N,) * 3, sp, H, dtype=dtype))
    return np.stack(out)


@pytest.fixture(scope="module")
def medium():
    vel = grf_velocity(N_PHYS, N_PHYS, N_PHYS, seed=41, corr_len=8.0)
    return vel, omega_for_ppw(float(vel.min()), H)


def _hier(vel, omega, precision, **kw):
    from paper_2608_22946_amd import helm
    return helm.Hierarchy(torch.from_numpy(vel), H, omega, NPML, precision=precision, table=load_iofd_table(),
                          device="cuda:0", tile_tz=8, tile_split=0, **kw)


@pytest.mark.parametrize("precision,batch,lanes", [("fp32", 4, 1), ("fp32", 2, 2), ("mixed", 3, 1), ("fp64", 5, 1)])
def test_batched_solve_equals_single_solves(medium, precision, batch, lanes):
    vel, omega = medium
    cdt = np.complex128 if precision == "fp64" else np.complex64
    f = torch.from_numpy(_sources(cdt)).cuda()
    one = _hier(vel, omega, precision)
    many = _hier(vel, omega, precision, batch=batch, lanes=lanes)
    u1, it1, rel1, rc1 = one.solve(f, 1e-6)
    ub, itb, relb, rcb = many.solve(f, 1e-6)
    torch.cuda.synchronize()
    print(f"\n{precision} batch {batch} lanes {lanes}: calls {list(itb)}")
    assert rc1 == 0 and rcb == 0
    assert list(it1) == list(itb) and np.array_equal(rel1, relb)
    assert torch.equal(u1, ub)
    assert itb[3] == 0 and float(ub[3].abs().max()) == 0.0
    assert len(set(int(i) for i in itb)) > 1   # the slots left the batch at different steps (the zero one at once)


def test_batched_solutions_match_oracle(medium):
    """Every right-hand side of an FP32 batch of four (plus a ragged group of one)
    against the oracle's converged solution."""
    from oracle.oracle import Hierarchy as OH
    vel, omega = medium
    f = _sources(np.complex64)
    g = _hier(vel, omega, "fp32", batch=4)
    u, its, relres, rc = g.solve(torch.from_numpy(f).cuda(), 1e-6)
    assert rc == 0 and np.all(relres <= 1e-6)
    o = OH(vel, H, omega, NPML, load_iofd_table())
    for k, sp in enumerate(SOURCES):
        if sp is None:
            continue
        uo, its_o, rel_o, st = o.solve(f[k].astype(np.complex128), 1e-10)
        assert st == 0
        err = rel(to_np(u[k]), uo)
        print(f"\nslot {k}: |u - u_ref| / |u_ref| = {err:.2e} ({int(its[k])} calls)")
        assert err <= 1e-5, (k, err)
    o.close()


def test_tuned_batch_tiling_matches_fixed_tiling(medium):
    """A batch whose stencil tiling setup times with all its slots running (the default)
    against the fixed tiling of the tests above: the same solutions up to the rounding
    order of the fused norms (the converged-solution bar)."""
    from paper_2608_22946_amd import helm
    vel, omega = medium
    f = torch.from_numpy(_sources(np.complex64)).cuda()
    fixed = _hier(vel, omega, "fp32", batch=4)
    tuned = helm.Hierarchy(torch.from_numpy(vel), H, omega, NPML, precision="fp32", table=load_iofd_table(),
                           device="cuda:0", batch=4)
    uf, itf, relf, rcf = fixed.solve(f, 1e-6)
    ut, itt, relt, rct = tuned.solve(f, 1e-6)
    assert rcf == 0 and rct == 0 and np.all(relt <= 1e-6)
    for k, sp in enumerate(SOURCES):
        if sp is None:
            assert float(ut[k].abs().max()) == 0.0
            continue
        err = rel(to_np(ut[k]), to_np(uf[k]))
        print(f"\nslot {k}: tuned vs fixed tiling {err:.2e} ({int(itt[k])} / {int(itf[k])} calls)")
        assert err <= 1e-5, (k, err)
