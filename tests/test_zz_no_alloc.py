"""The allocation-free projection (fbto_project_volume_noalloc) against the
grid-handle projection (fbto_project_volume) it shares its kernels with:
two calls in a row on one GPU, the second on a smaller input, each checked
bit for bit against the handle's result and against the KKT conditions of
Sec. 4.2 (x = clamp(y - lambda, lo, hi), sum x = vmax when active)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, say

pytestmark = pytest.mark.gpu


def _case(E, seed, dtype):
    rng = np.random.default_rng(seed)
    y = rng.uniform(-0.3, 1.4, E)
    vmax = 0.3 * E
    return torch.tensor(y, dtype=dtype, device=DEV), vmax


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_projection_matches_the_handle_projection(dtype):
    from paper_2204_06204_amd.grid import Grid, project_volume_noalloc
    sizes = [(64, 32, 32), (20, 9, 7)]  # second call: smaller input
    for i, (nx, ny, nz) in enumerate(sizes):
        E = nx * ny * nz
        say(f"noalloc projection: call {i}, E = {E}, {dtype}")
        y, vmax = _case(E, 10 + i, dtype)
        g = Grid(nx, ny, nz, filter_radius=1.0)
        lam_r = torch.zeros(1, dtype=torch.float64, device=DEV)
        st_r = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
        x_ref = g.project_volume(y, lo=0.0, hi=1.0, vmax=vmax, lam=lam_r, status=st_r, max_passes=16)
        lam = torch.zeros(1, dtype=torch.float64, device=DEV)
        st = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
        x = project_volume_noalloc(y, lo=0.0, hi=1.0, vmax=vmax, max_passes=16, lam=lam, status=st)
        xr, xa = host(x_ref), host(x)
        assert float(host(st)[0]) == 0.0 and float(host(st_r)[0]) == 0.0
        assert np.array_equal(xa, xr), "not bitwise equal to fbto_project_volume"
        assert float(host(lam)[0]) == float(host(lam_r)[0])
        # KKT of the projection, from the host copy of y
        yh = host(y)
        lm = float(host(lam)[0])
        assert lm > 0.0
        want = np.clip(yh - lm, 0.0, 1.0)
        tol = 1e-12 if dtype == torch.float64 else 1e-6
        assert np.max(np.abs(xa - want)) <= tol
        assert abs(xa.sum() - vmax) <= (1e-9 if dtype == torch.float64 else 2e-3) * vmax
        g.close()
