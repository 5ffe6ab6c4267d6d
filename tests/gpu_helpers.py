"""Shared helpers of the GPU parity tests: seeded problems on both sides."""
import numpy as np

from paper_2008_00409_amd import meshgen as mg


def require_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def sheet(nx, ny, seed=7, ell=0.02, flips=0.0, bumps=True, h=0.01, delaunay=True):
    """Irregular sheet with a pinned top row, lumped mass (nx*ny vertices)."""
    rest, tris, pinned, x0 = mg.irregular_sheet(nx, ny, ell, 0.0, seed, flips, bumps=bumps, delaunay=delaunay)
    mass = mg.lumped_mass(rest, tris, mg.AREAL_DENSITY)
    return mg.Cloth(f"sheet-{nx}x{ny}", rest, tris, mass, pinned, x0, np.zeros_like(rest), h, 1e-6, 1,
                    [(0, rest.shape[0])], [(0, tris.shape[0])])


def random_velocity(c, scale=0.05, seed=3):
    v = scale * np.random.default_rng(seed).normal(size=c.rest.shape)
    v[c.pinned == 1] = 0.0
    return v


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def block_rel_err(got, want):
    """Max over blocks of |got - want| / (max |want| in that block's row)."""
    return float(np.max(np.abs(got - want)))
