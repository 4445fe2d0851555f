"""GPU: the batching configuration's stopping rule, max|drho| < 1e-9 per step, reached
by the batched solver.  The cases are the Carnahan-Starling cases of at most 256
columns from the 256-case batching draw (side 128-512, Tr 0.6-0.9, drop radius a
quarter of the side on a CP wall), in FP64 storage: FP32 storage cannot get there
(its rounding keeps the field moving at a few 1e-8 per step).  Measured: all 33 stop
within 9000-51000 steps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")
from paper_1611_00907_amd import inputs  # noqa: E402

import bench  # noqa: E402


def test_fp64_batch_reaches_the_residual_and_conserves_mass():
    params, rhos, muw = bench.batch_workload(lbm, inputs)
    sel = [k for k, p in enumerate(params) if p.eos == lbm.LBM_EOS_CS and p.nx <= 256]
    assert len(sel) >= 30
    ps = []
    for k in sel:
        p = params[k]
        p.prec = lbm.LBM_F64
        ps.append(p)
    b = lbm.Batch(ps, [rhos[k] for k in sel], mu_w_bottom=[muw[k] for k in sel])
    b.run(70000, check_every=1000, window=1000, tol=1e-9)
    st = b.status()
    m0 = np.array([rhos[k][1:-1].sum() for k in sel])
    b.close()
    print("steps to the residual: median %d, max %d" % (np.median(st["steps"]), st["steps"].max()))
    assert (st["state"] == 1).all(), st["state"]
    assert (st["residual"] < 1e-9).all()
    # halfway bounce-back and the Eq 28 ghost rows move no mass across the walls
    np.testing.assert_allclose(st["mass"], m0, rtol=1e-11)
