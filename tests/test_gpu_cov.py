"""GPU parity of the covariance -> steps mapping (bsf_cov_to_steps) against
the oracle: minimum-kurtosis steps of both four-direction box splines, order 1
and tied order 2, the isotropic rule, an Alg. 1-style diagonal shift, and the
range flag for covariances out of reach."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def cov_field(rng, H, W, rho_max=None, bank=1, sig=(1.5, 12.0)):
    """Smooth orientation, elongation and size fields -> C11, C12, C22."""
    th = WL.smooth(rng, H, W, 0.0, np.pi)
    rho = WL.smooth(rng, H, W, 1.0, 4.0 if rho_max is None else rho_max)
    if bank == 1 and rho_max is None:
        rho = np.minimum(rho, 0.9 * np.array([[O.elongation_bound(t) for t in row] for row in th]))
    sig = WL.smooth(rng, H, W, *sig)
    l1, l2 = sig ** 2, sig ** 2 / rho
    c, s = np.cos(th), np.sin(th)
    C11 = l1 * c * c + l2 * s * s
    C22 = l1 * s * s + l2 * c * c
    C12 = (l1 - l2) * c * s
    return np.stack([C11, C12, C22]).astype(np.float32)


def gpu_steps(cfg, cov, sub=0.0):
    ws = bsf.Workspace(256, DEV)
    st = bsf.cov_to_steps(cfg, torch.from_numpy(cov).to(DEV), sub=sub, ws=ws)
    flags, _, _ = ws.status()
    return st.cpu().numpy(), flags


def kurt(dirs, steps):
    A = steps.astype(np.float64) ** 2 / 12.0
    K = np.zeros((3,) + steps.shape[1:])
    for k, (ux, uy) in enumerate(dirs):
        n2 = ux * ux + uy * uy
        K[0] += A[k] ** 2 * n2 * ux * ux
        K[1] += A[k] ** 2 * n2 * ux * uy
        K[2] += A[k] ** 2 * n2 * uy * uy
    return K[0] ** 2 + 2 * K[1] ** 2 + K[2] ** 2


@pytest.mark.parametrize("bank,order", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_cov_to_steps_matches_oracle(bank, order):
    note("cov->steps bank", bank, "order", order)
    rng = np.random.default_rng(200 + 10 * bank + order)
    dirs = O.BANK1 if bank == 1 else O.BANK2
    H, W = 96, 130
    cov = cov_field(rng, H, W, bank=bank, rho_max=3.0 if bank == 2 else None)
    cfg = bsf.Config(dirs=dirs, order=order, max_step=200.0)
    got, flags = gpu_steps(cfg, cov)
    ref, rflags = O.cov_to_steps_field(dirs, order, cov)
    assert flags == 0 and not rflags.any()
    # the minimiser of a quartic can be flat: compare the steps, and where they
    # differ more than rounding, the objective they reach must be as low
    close = np.isclose(got, ref, rtol=2e-6, atol=0)
    far = ~close.all(axis=0)
    assert far.mean() < 0.01, far.mean()
    kg, kr = kurt(dirs, got[:, far]), kurt(dirs, ref[:, far])
    assert (kg <= kr * (1 + 1e-6)).all()
    # the covariance is reproduced wherever no step is at its floor
    A = got.astype(np.float64) ** 2 / 12.0 * order
    C = np.zeros((3, H, W))
    for k, (ux, uy) in enumerate(dirs):
        C[0] += A[k] * ux * ux
        C[1] += A[k] * ux * uy
        C[2] += A[k] * uy * uy
    free = (got > 1.0).all(axis=0)
    assert free.mean() > 0.3
    np.testing.assert_allclose(C[:, free], cov[:, free].astype(np.float64), rtol=2e-6, atol=2e-5)


def test_cov_to_steps_isotropic_and_shift():
    """C = sigma^2 I gives sqrt(6) sigma physical scales; subtracting sub from
    the diagonal equals passing C - sub I."""
    note("cov->steps isotropic / shift")
    H, W = 8, 9
    sig = np.linspace(1.0, 9.0, H * W).reshape(H, W)
    cov = np.stack([sig ** 2, np.zeros_like(sig), sig ** 2]).astype(np.float32)
    cfg = bsf.Config(order=1, max_step=200.0)
    got, flags = gpu_steps(cfg, cov)
    assert flags == 0
    np.testing.assert_allclose(got[0], np.maximum(np.sqrt(6) * sig, 1), rtol=1e-6)
    np.testing.assert_allclose(got[2], np.maximum(np.sqrt(3) * sig, 1), rtol=1e-6)
    rng = np.random.default_rng(230)
    cov = cov_field(rng, 40, 50)
    shifted = cov.copy()
    shifted[0] -= 1.5
    shifted[2] -= 1.5
    a, _ = gpu_steps(cfg, cov, sub=1.5)
    b, _ = gpu_steps(cfg, shifted)
    np.testing.assert_allclose(a, b, rtol=1e-6)


def test_cov_out_of_reach_is_flagged():
    note("cov->steps out of reach")
    phi = np.deg2rad(22.5)
    R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    C = R @ np.diag([50.0, 50.0 / 8.0]) @ R.T        # elongation 8 > 5.83
    cov = np.zeros((3, 4, 4), np.float32)
    cov[0], cov[1], cov[2] = C[0, 0], C[0, 1], C[1, 1]
    cov[1, 2, 2] = np.nan
    got, flags = gpu_steps(bsf.Config(order=1, max_step=200.0), cov)
    assert flags & bsf.FLAG_RANGE
    assert (got >= 1.0).all() and np.isfinite(got).all()
    ref, rflag = O.cov_to_steps(O.BANK1, 1, C[0, 0], C[0, 1], C[1, 1])
    assert rflag
    np.testing.assert_allclose(got[:, 0, 0], ref, rtol=1e-5)
