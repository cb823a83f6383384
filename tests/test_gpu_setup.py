"""Per-element block inverses built on the GPU (assembled from n_b colour
residuals of unit vectors, FP64 Gauss-Jordan with partial pivoting on the
equilibrated block, written into the tile layout of each precision) against
the host build (LDGS_DEVICE_SETUP=0: host assembly, equilibrated LU, explicit
inverse): colour passes on every smoothed level and colour in FP64, FP32 and
with BF16-stored inverses, and V-cycle residual histories."""
import numpy as np
import pytest

from synth import Problem, SinProductField, c2_dirichlet_varmu, c4a_square_inclusion, c5_lognormal

pytestmark = pytest.mark.gpu

CASES = {
    "c2_n16_p3": lambda: c2_dirichlet_varmu(n=16, p=3),
    "c2_n16_p1": lambda: c2_dirichlet_varmu(n=16, p=1),
    "c4a_n16_p2": lambda: c4a_square_inclusion(n=16, p=2),
    "c5_n8_p2": lambda: c5_lognormal(n=8, p=2),
    "c5_n8_p2_scaled": lambda: c5_lognormal(n=8, p=2, diag_scaling=True),
    "dir3d_n8_p1_std": lambda: Problem(name="d3", dim=3, n=8, p=1, gamma=0, bc=("dirichlet",) * 3,
                                       mu=SinProductField(1.0, 0.5, 2.0)),
    "unsteady_dir2d_n16_p2": lambda: Problem(name="u", dim=2, n=16, p=2, gamma=1, bc=("dirichlet",) * 2,
                                             mu=__import__("synth").ConstField(1.0),
                                             rho=__import__("synth").ConstField(1.0), delta=1e-3),
}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_device_inverses_match_host_build(name, monkeypatch):
    import torch
    from paper_1911_05888_amd import Context, V_FP32, V_FP32_BF16BLK
    prob = CASES[name]()
    print(f"[setup] device vs host inverses {name}", flush=True)
    ctxs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("LDGS_DEVICE_SETUP", flag)
        ctxs.append(Context(prob, build_precisions=(1 << V_FP32) | (1 << V_FP32_BF16BLK)))
    dev, host = ctxs
    rng = np.random.Generator(np.random.PCG64(61))
    worst = {0: 0.0, 1: 0.0, 2: 0.0}
    for l in range(dev.n_levels - 1):
        if dev.level_shared_inverse(l):
            continue
        n_l, _, ncol = dev.level_info(l)
        N = n_l ** prob.dim * prob.nb
        x0, b = rng.standard_normal(N), rng.standard_normal(N)
        xd = torch.tensor(x0, device="cuda")
        xh = xd.clone()
        bg = torch.tensor(b, device="cuda")
        for c in range(ncol):
            dev.level_smooth_colour(l, c, bg, xd)
            host.level_smooth_colour(l, c, bg, xh)
            worst[0] = max(worst[0], _rel(xd.cpu().numpy(), xh.cpu().numpy()))
        for vp in (V_FP32, V_FP32_BF16BLK):
            xd = torch.tensor(x0, dtype=torch.float32, device="cuda")
            xh = xd.clone()
            b32 = bg.float()
            for c in range(ncol):
                dev.level_smooth_colour_f32(l, c, vp, b32, xd)
                host.level_smooth_colour_f32(l, c, vp, b32, xh)
            worst[vp] = max(worst[vp], _rel(xd.double().cpu().numpy(), xh.double().cpu().numpy()))
    print(f"[setup]   colour passes FP64 {worst[0]:.2e} FP32 {worst[1]:.2e} BF16-inverse {worst[2]:.2e}", flush=True)
    assert worst[0] <= 1e-11 and worst[1] <= 1e-5 and worst[2] <= 1e-2, worst
    # FP64 V-cycle histories
    bh = rng.standard_normal(dev.ndof)
    hists = []
    for ctx in (dev, host):
        b = torch.tensor(bh, device="cuda")
        x = torch.zeros_like(b)
        st, info = ctx.solve(b, x, tol=0.0, maxit=6)
        hists.append(info["history"])
    assert np.abs(hists[0] - hists[1]).max() <= 1e-11 * max(1.0, hists[1].max()), (hists[0], hists[1])
