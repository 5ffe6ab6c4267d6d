"""Seeded synthetic cloth inputs.

This module only builds inputs: rest positions, triangles, masses, pin flags,
initial positions and velocities.  It contains none of the integrator's
arithmetic (no strain, force, Jacobian, assembly or solve), so both the FP64
oracle and the HIP path can take their inputs from it without sharing any of
the method.

The paper's benchmark garments are not available; the workloads below are
synthetic stand-ins with the paper's sizes (0.5M-1.65M triangles, several
pieces of cloth, irregular meshes; Sec. 5 benchmark list).

Conventions
-----------
* Grid vertex (i, j) has id ``j*nx + i`` and rest position ``(i*dx, j*dy, z0)``.
* Quad ``q = j*(nx-1) + i`` is split into triangles ``2q = (v00, v10, v11)``
  and ``2q+1 = (v00, v11, v01)``, counter-clockwise seen from +z.
* Positions are returned as (nv, 3) float64 arrays, triangles as (nt, 3) int32.
* Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)
MU = 1000.0          # N/m, membrane shear modulus (StVK reading of the stretch law)
LAMBDA = 500.0       # N/m, membrane Lame constant
K_BEND = 1e-5        # N*m, dihedral bending stiffness
AREAL_DENSITY = 0.2  # kg/m^2, lumped mass for the large workloads


@dataclasses.dataclass
class Cloth:
    """One cloth problem: topology, rest shape, masses, pins and initial state."""
    name: str
    rest: np.ndarray      # (nv, 3) float64 rest positions X
    tris: np.ndarray      # (nt, 3) int32, CCW w.r.t. +z
    mass: np.ndarray      # (nv,) float64, kg
    pinned: np.ndarray    # (nv,) uint8, 1 = Dirichlet vertex
    x0: np.ndarray        # (nv, 3) float64 initial positions
    v0: np.ndarray        # (nv, 3) float64 initial velocities
    h: float              # time step, s
    tol: float            # CG relative residual target
    steps: int            # steps in the workload
    sheet_ranges: list    # [(vertex_begin, vertex_end)] per disconnected sheet/instance
    tri_ranges: list      # [(tri_begin, tri_end)] per sheet/instance

    @property
    def nv(self) -> int:
        return int(self.rest.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid(nx: int, ny: int, width: float, height: float, z0: float = 0.0):
    """Regular nx-by-ny vertex grid spanning width x height in the plane z = z0."""
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    rest = np.zeros((nx * ny, 3), dtype=np.float64)
    rest[:, 0] = (ii.ravel() * (width / (nx - 1)))
    rest[:, 1] = (jj.ravel() * (height / (ny - 1)))
    rest[:, 2] = z0
    qi, qj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    qi = qi.ravel()
    qj = qj.ravel()
    v00 = qj * nx + qi
    v10 = v00 + 1
    v01 = v00 + nx
    v11 = v01 + 1
    tris = np.empty((2 * qi.size, 3), dtype=np.int32)
    tris[0::2] = np.stack([v00, v10, v11], axis=1)
    tris[1::2] = np.stack([v00, v11, v01], axis=1)
    return rest, tris


def lumped_mass(rest: np.ndarray, tris: np.ndarray, density: float) -> np.ndarray:
    """Each vertex receives a third of the rest area of every incident triangle."""
    a = rest[tris[:, 1]] - rest[tris[:, 0]]
    b = rest[tris[:, 2]] - rest[tris[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(a, b), axis=1)
    m = np.zeros(rest.shape[0], dtype=np.float64)
    for k in range(3):
        np.add.at(m, tris[:, k], density * area / 3.0)
    return m


def jitter_rest(rest: np.ndarray, nx: int, ny: int, ell: float, frac: float,
                rng: np.random.Generator) -> np.ndarray:
    """Move non-boundary grid vertices in-plane, uniformly inside a disk of radius frac*ell."""
    out = rest.copy()
    ii = np.arange(nx * ny) % nx
    jj = np.arange(nx * ny) // nx
    inner = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1)
    n = int(inner.sum())
    r = frac * ell * np.sqrt(rng.random(n))
    phi = 2.0 * math.pi * rng.random(n)
    out[inner, 0] += r * np.cos(phi)
    out[inner, 1] += r * np.sin(phi)
    return out


def interior_edges(tris: np.ndarray):
    """Interior edges as (a, b, t1, t2): t1 holds directed edge a->b, t2 holds b->a."""
    nt = tris.shape[0]
    src = tris.reshape(-1)
    dst = tris[:, [1, 2, 0]].reshape(-1)
    tri_of = np.repeat(np.arange(nt), 3)
    lo = np.minimum(src, dst).astype(np.int64)
    hi = np.maximum(src, dst).astype(np.int64)
    key = lo * (int(src.max()) + 1) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    e0 = order[same]
    e1 = order[same + 1]
    # e0 is a directed edge src->dst of triangle tri_of[e0]
    a = src[e0]
    b = dst[e0]
    return a, b, tri_of[e0], tri_of[e1]


def flip_edges(rest: np.ndarray, tris: np.ndarray, fraction: float,
               rng: np.random.Generator, delaunay: bool = True, strict: bool = False) -> np.ndarray:
    """Flip a random `fraction` of interior edges.

    A flip of edge a-b between t1=(a,b,c) and t2=(b,a,d) replaces them with
    (c,a,d) and (d,b,c).  With `delaunay` (the default) only illegal edges are
    flipped -- d strictly inside the circumcircle of (a,b,c) in the rest plane --
    so every flip makes its edge Delaunay-legal (and the quad is then convex).
    A flip is accepted only when both new triangles have positive area, the new
    diagonal c-d is not already an edge, and neither triangle has been flipped
    before in this pass.  Edges are visited in a seeded random order until the
    target count is reached (or every edge has been visited; `strict` then
    raises).
    """
    tris = tris.copy()
    a, b, t1, t2 = interior_edges(tris)
    target = int(round(fraction * a.size))
    nv = rest.shape[0]
    e_src = tris.reshape(-1).astype(np.int64)
    e_dst = tris[:, [1, 2, 0]].reshape(-1).astype(np.int64)
    edges = set((np.minimum(e_src, e_dst) * nv + np.maximum(e_src, e_dst)).tolist())
    used = np.zeros(tris.shape[0], dtype=bool)
    perm = rng.permutation(a.size)
    xy = rest[:, :2]

    def third(t, p, q):
        row = tris[t]
        for w in row:
            if w != p and w != q:
                return int(w)
        return -1

    def ccw(p, q, r):
        return ((xy[q, 0] - xy[p, 0]) * (xy[r, 1] - xy[p, 1])
                - (xy[q, 1] - xy[p, 1]) * (xy[r, 0] - xy[p, 0]))

    def in_circle(p, q, r, t):
        # > 0 when t lies inside the circumcircle of the counter-clockwise p, q, r
        rows = []
        for u in (p, q, r):
            dx, dy = xy[u, 0] - xy[t, 0], xy[u, 1] - xy[t, 1]
            rows.append((dx, dy, dx * dx + dy * dy))
        (a1, a2, a3), (b1, b2, b3), (c1, c2, c3) = rows
        return a1 * (b2 * c3 - b3 * c2) - a2 * (b1 * c3 - b3 * c1) + a3 * (b1 * c2 - b2 * c1)

    done = 0
    for e in perm:
        if done >= target:
            break
        ta, tb = int(t1[e]), int(t2[e])
        if used[ta] or used[tb]:
            continue
        va, vb = int(a[e]), int(b[e])
        c = third(ta, va, vb)
        d = third(tb, va, vb)
        if c == d:
            continue
        key = min(c, d) * nv + max(c, d)
        if key in edges:
            continue
        if ccw(c, va, d) <= 0.0 or ccw(d, vb, c) <= 0.0:
            continue
        if delaunay and in_circle(va, vb, c, d) <= 0.0:
            continue
        tris[ta] = (c, va, d)
        tris[tb] = (d, vb, c)
        used[ta] = used[tb] = True
        edges.discard(min(va, vb) * nv + max(va, vb))
        edges.add(key)
        done += 1
    if done < target and strict:
        raise RuntimeError(f"edge flips: reached {done} of {target}")
    return tris


def gaussian_bumps(rest: np.ndarray, rng: np.random.Generator, extent, n: int = 8) -> np.ndarray:
    """Out-of-plane displacement: sum of n Gaussians, amplitudes +-U(0.01, 0.05) m,
    centres uniform over the sheet's extent, widths U(0.05, 0.15) m."""
    (x_lo, x_hi), (y_lo, y_hi) = extent
    amp = rng.uniform(0.01, 0.05, n) * rng.choice([-1.0, 1.0], n)
    cx = rng.uniform(x_lo, x_hi, n)
    cy = rng.uniform(y_lo, y_hi, n)
    sig = rng.uniform(0.05, 0.15, n)
    dz = np.zeros(rest.shape[0])
    for k in range(n):
        r2 = (rest[:, 0] - cx[k]) ** 2 + (rest[:, 1] - cy[k]) ** 2
        dz += amp[k] * np.exp(-r2 / (2.0 * sig[k] ** 2))
    return dz


def config_tiny(seed: int = 1000) -> Cloth:
    """32x32-vertex square, 1 m x 1 m, top corners pinned, 1e-3 kg per vertex,
    positions jittered by U(-1e-3, 1e-3) m (non-pinned vertices), h = 0.01 s,
    tolerance 1e-8.  1,024 vertices, 1,922 triangles."""
    nx = ny = 32
    rest, tris = grid(nx, ny, 1.0, 1.0)
    nv = rest.shape[0]
    pinned = np.zeros(nv, dtype=np.uint8)
    pinned[[992, 1023]] = 1
    mass = np.full(nv, 1e-3)
    rng = _rng(seed)
    x0 = rest + rng.uniform(-1e-3, 1e-3, size=rest.shape) * (1 - pinned)[:, None]
    return Cloth("tiny-32x32", rest, tris, mass, pinned, x0, np.zeros_like(rest),
                 0.01, 1e-8, 1, [(0, nv)], [(0, tris.shape[0])])


def config_grid(n: int, seed: int = 2000, h: float = 1.0 / 200, tol: float = 1e-6,
                steps: int = 200, name: str | None = None) -> Cloth:
    """n x n-vertex square, 1 m x 1 m, top row pinned, areal density 0.2 kg/m^2,
    flat rest, initial positions = rest + 8 seeded Gaussian bumps (1-5 cm).
    n = 512 is the medium workload: 262,144 vertices, 522,242 triangles."""
    rest, tris = grid(n, n, 1.0, 1.0)
    nv = rest.shape[0]
    pinned = np.zeros(nv, dtype=np.uint8)
    pinned[(n - 1) * n:] = 1
    mass = lumped_mass(rest, tris, AREAL_DENSITY)
    rng = _rng(seed)
    x0 = rest.copy()
    x0[:, 2] += gaussian_bumps(rest, rng, ((0.0, 1.0), (0.0, 1.0)))
    return Cloth(name or f"grid-{n}x{n}", rest, tris, mass, pinned, x0, np.zeros_like(rest),
                 h, tol, steps, [(0, nv)], [(0, tris.shape[0])])


def config_medium(seed: int = 2000) -> Cloth:
    return config_grid(512, seed=seed, name="medium-512x512")


def irregular_sheet(nx: int, ny: int, ell: float, z0: float, seed: int,
                    flip_fraction: float, bumps: bool = True, strict: bool = False,
                    delaunay: bool = True):
    """Jittered (0.3 ell, in-plane, interior vertices) and edge-flipped grid sheet
    with its top row pinned; returns rest, tris, pinned, initial positions."""
    rng = _rng(seed)
    width, height = ell * (nx - 1), ell * (ny - 1)
    rest, tris = grid(nx, ny, width, height, z0)
    rest = jitter_rest(rest, nx, ny, ell, 0.3, rng)
    if flip_fraction > 0.0:
        tris = flip_edges(rest, tris, flip_fraction, rng, delaunay=delaunay, strict=strict)
    pinned = np.zeros(rest.shape[0], dtype=np.uint8)
    pinned[(ny - 1) * nx:] = 1
    x0 = rest.copy()
    if bumps:
        x0[:, 2] += gaussian_bumps(rest, rng, ((0.0, width), (0.0, height)))
    return rest, tris, pinned, x0


def stack_sheets(parts, name, h, tol, steps) -> Cloth:
    rests, triss, pins, xs = [], [], [], []
    vranges, tranges = [], []
    off = 0
    toff = 0
    for rest, tris, pinned, x0 in parts:
        rests.append(rest)
        triss.append(tris + off)
        pins.append(pinned)
        xs.append(x0)
        vranges.append((off, off + rest.shape[0]))
        tranges.append((toff, toff + tris.shape[0]))
        off += rest.shape[0]
        toff += tris.shape[0]
    rest = np.concatenate(rests)
    tris = np.concatenate(triss).astype(np.int32)
    mass = lumped_mass(rest, tris, AREAL_DENSITY)
    x0 = np.concatenate(xs)
    return Cloth(name, rest, tris, mass, np.concatenate(pins), x0, np.zeros_like(rest),
                 h, tol, steps, vranges, tranges)


def config_large(seed_base: int = 3000, sheets: int = 3, nx: int = 501, ny: int = 551,
                 flip_fraction: float = 0.10) -> Cloth:
    """Three stacked irregular sheets, 501 x 551 vertices each (550,000 triangles
    each, 1.65M in total), edge length 2 mm, at z = 0, 0.02, 0.04 m; 10% of
    interior edges flipped; top rows pinned; h = 0.01 s, tolerance 1e-6."""
    parts = [irregular_sheet(nx, ny, 0.002, 0.02 * s, seed_base + s, flip_fraction, strict=True)
             for s in range(sheets)]
    return stack_sheets(parts, f"stacked-{sheets}x{nx}x{ny}", 0.01, 1e-6, 100)


def batch_sizes(count: int = 64, seed: int = 5000):
    """Triangle targets log-uniform in [2e3, 1e5]; each instance is a square
    grid with round(sqrt(T/2)) + 1 vertices per side."""
    rng = _rng(seed)
    t = np.round(np.exp(rng.uniform(math.log(2e3), math.log(1e5), count))).astype(np.int64)
    return [int(round(math.sqrt(tk / 2.0))) + 1 for tk in t]


def config_batch(count: int = 64, seed: int = 5000, sizes=None) -> Cloth:
    """Many independent square sheets (1 m wide, jittered, no flips, top row pinned,
    bumps) concatenated into one vertex/triangle range each."""
    sides = sizes if sizes is not None else batch_sizes(count, seed)
    parts = []
    for k, n in enumerate(sides):
        ell = 1.0 / (n - 1)
        parts.append(irregular_sheet(n, n, ell, 0.0, seed + 1 + k, 0.0))
    return stack_sheets(parts, f"batch-{len(sides)}", 0.01, 1e-6, 100)


@dataclasses.dataclass
class ContactSet:
    """Proximity pairs handed to the solver for one step: vertices (nc, 4),
    weights (nc, 4) summing to zero per pair, unit normals (nc, 3), thickness
    eta (m) and stiffness kc (N/m)."""
    verts: np.ndarray
    weights: np.ndarray
    normals: np.ndarray
    eta: float
    kc: float

    @property
    def n(self) -> int:
        return int(self.verts.shape[0])


def vf_contacts(x: np.ndarray, tris: np.ndarray, verts, tri_ids, radius: float, eta: float, kc: float,
                candidates: int = 6) -> ContactSet:
    """Vertex-face proximity pairs, as a collision query would report them:
    each vertex of `verts` is paired with the first of its `candidates`
    nearest triangles of `tri_ids` (by centroid) onto whose plane it projects
    inside the triangle within `radius`.  Weights (1, -w_a, -w_b, -w_c) are the
    projection's barycentric coordinates, the normal is the triangle's unit
    normal turned towards the vertex."""
    from scipy.spatial import cKDTree
    verts = np.asarray(verts, dtype=np.int64)
    tri_ids = np.asarray(tri_ids, dtype=np.int64)
    T = tris[tri_ids]
    a, b, c = x[T[:, 0]], x[T[:, 1]], x[T[:, 2]]
    cen = (a + b + c) / 3.0
    tree = cKDTree(cen)
    _, cand = tree.query(x[verts], k=min(candidates, len(tri_ids)))
    cand = np.atleast_2d(cand)
    P = x[verts][:, None, :]                                  # (n, 1, 3)
    A, B, C = a[cand], b[cand], c[cand]                       # (n, k, 3)
    nrm = np.cross(B - A, C - A)
    ln = np.linalg.norm(nrm, axis=2, keepdims=True)
    ok = ln[..., 0] > 0.0
    nrm = nrm / np.where(ln > 0.0, ln, 1.0)
    d = np.einsum("nka,nka->nk", P - A, nrm)
    sgn = np.where(d < 0.0, -1.0, 1.0)
    nrm = nrm * sgn[..., None]
    d = d * sgn
    q = P - d[..., None] * nrm
    v0, v1, v2 = B - A, C - A, q - A
    d00 = np.einsum("nka,nka->nk", v0, v0)
    d01 = np.einsum("nka,nka->nk", v0, v1)
    d11 = np.einsum("nka,nka->nk", v1, v1)
    d20 = np.einsum("nka,nka->nk", v2, v0)
    d21 = np.einsum("nka,nka->nk", v2, v1)
    den = d00 * d11 - d01 * d01
    ok &= den > 0.0
    den = np.where(ok, den, 1.0)
    wb = (d11 * d20 - d01 * d21) / den
    wc = (d00 * d21 - d01 * d20) / den
    wa = 1.0 - wb - wc
    ok &= (d < radius) & (wa >= 0.0) & (wb >= 0.0) & (wc >= 0.0)
    has = ok.any(axis=1)
    first = np.argmax(ok, axis=1)                               # first valid candidate
    rows = np.nonzero(has)[0]
    k = first[rows]
    t = T[cand[rows, k]]
    cverts = np.column_stack([verts[rows], t]).astype(np.int32)
    weights = np.column_stack([np.ones(rows.size), -wa[rows, k], -wb[rows, k], -wc[rows, k]])
    return ContactSet(cverts, weights, nrm[rows, k], eta, kc)


def config_contact(nx: int = 501, ny: int = 551, gap: float = 0.0015, seed_base: int = 6000) -> tuple:
    """Two irregular sheets (2 mm edges, 10% flips, same bumps) with the upper
    one `gap` above the lower, top rows pinned, h = 0.01 s; returns the cloth
    and the vertex-face pairs of every upper vertex within the thickness
    eta = 2 mm of the lower sheet (kc = 1000 N/m)."""
    lower = irregular_sheet(nx, ny, 0.002, 0.0, seed_base, 0.10, strict=True)
    upper = irregular_sheet(nx, ny, 0.002, gap, seed_base + 1, 0.10, strict=True)
    # the same bumps on both sheets, so the gap is uniform
    bump = lower[3][:, 2] - lower[0][:, 2]
    rest_u, tris_u, pin_u, _ = upper
    x_u = rest_u.copy()
    x_u[:, 2] += _bump_at(lower[0], bump, rest_u)
    c = stack_sheets([lower, (rest_u, tris_u, pin_u, x_u)], f"contact-2x{nx}x{ny}", 0.01, 1e-6, 100)
    nl = lower[0].shape[0]
    cs = vf_contacts(c.x0, c.tris, np.arange(nl, c.nv), np.arange(0, lower[1].shape[0]), 0.002, 0.002, 1000.0)
    return c, cs


def _bump_at(rest_lower: np.ndarray, bump_lower: np.ndarray, points: np.ndarray) -> np.ndarray:
    """The lower sheet's bump height at the nearest lower rest vertex of each point."""
    from scipy.spatial import cKDTree
    _, idx = cKDTree(rest_lower[:, :2]).query(points[:, :2])
    return bump_lower[idx]


def mesh_counts(tris: np.ndarray, nv: int):
    """(interior edges, distinct off-diagonal block pairs) from topology alone:
    used to check the generators against the expected sizes."""
    a, b, t1, t2 = interior_edges(tris)
    return int(a.size)
