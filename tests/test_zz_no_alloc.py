"""The static-workspace binding (hhg_bind_static_workspace, for callers that cannot allocate)
against the torch-allocated one (hhg_bind_workspace): the same solve and estimate on two
contexts bound one after the other, the second smaller, at the parity bar (1e-12 of the
solution for u, 1e-12 * ||u|| for estimator quantities)."""
import numpy as np
import pytest

from gpu_common import to_dev, to_host
from workloads import meshes, problems

pytestmark = pytest.mark.gpu


def _data(name, X):
    if name == "lshape":
        return np.zeros(len(X)), problems.lshape_u(X)
    return problems.sine2d_f(X), np.zeros(len(X))


def _run(hh, f, g):
    u, st = hh.fmg_solve(f, g, nu=1, pre=2, post=2, rtol=0.0, max_iter=2)
    est = hh.estimate(1)
    return to_host(u), est, st


def test_static_workspace_matches_torch_workspace():
    from paper_2508_06049_amd import HHG, HHGError
    from paper_2508_06049_amd._lib import HHG_ENOMEM, HHG_ESTATE

    cases = [("lshape", meshes.lshape_6tri(), 6, "multicolour"), ("square", meshes.unit_square_2tri(), 4, "redblack")]
    prev = None
    for name, m, L, sm in cases:
        print(f"[case] static workspace {name} L={L}", flush=True)
        ref = HHG(m.coords, m.cells, L, smoother=sm)
        X = to_host(ref.dof_coords())
        f, g = _data(name, X)
        fd, gd = to_dev(f), to_dev(g)
        ur, er, sr = _run(ref, fd, gd)
        hs = HHG(m.coords, m.cells, L, smoother=sm, workspace="static")
        if prev is not None:
            # the earlier context lost the array to this one
            hp, fp, gp = prev
            with pytest.raises(HHGError) as ei:
                hp.fmg_solve(fp, gp, nu=1)
            assert ei.value.status == HHG_ESTATE
        for rep in range(2):
            us, es, ss = _run(hs, fd, gd)
            scale = np.abs(ur).max()
            assert np.abs(us - ur).max() <= 1e-12 * scale
            tol = 1e-12 * np.sqrt(float(ur @ to_host(ref.mass_apply(to_dev(ur)))))
            assert np.abs(es["eta_T"] - er["eta_T"]).max() <= tol
            assert abs(es["norm_e"] - er["norm_e"]) <= tol
            assert ss.vcycles == sr.vcycles and ss.ms_total == 0.0
        ref.close()
        prev = (hs, fd, gd)
    prev[0].close()
    # a context larger than the static array is refused
    m = meshes.lshape_6tri()
    with pytest.raises(HHGError) as ei:
        HHG(m.coords, m.cells, 10, smoother="multicolour", workspace="static")
    assert ei.value.status == HHG_ENOMEM
