"""Seeded synthetic scene generators.

These build the inputs of the mass-spring method (masses, springs, their
parameters and per-spring actuation) for both the native GPU path and the
FP64 reference used by the tests.  They hold none of the stepping arithmetic:
no forces, no rest lengths, no integration.  Every random draw comes from a
``numpy.random.Generator(PCG64(seed))`` in a fixed, documented order so that a
scene is a pure function of its arguments.

Scenes are returned as plain dicts of numpy arrays in the layout the C ABI
takes:

* ``pos``     (n, 3) float32, metres
* ``vel``     (n, 3) float32, m/s
* ``mass``    (n,)   float32, kg (0 marks a pinned mass)
* ``ends``    (s, 2) int64, mass indices of each spring
* ``k``       (s,)   float32, N/m
* ``damping`` (s,)   float32, N*s/m
* ``amp``, ``phase`` (s,) float32 or None: actuation, the rest length being
  scaled by ``1 + amp * sin(omega * t + phase)`` (the paper's actuation law,
  Sec. IV-B Eq. 4, with a per-spring phase in place of its time offset)
* ``body``    (n,) int32 or None, index of the independent body of each mass

The lattice rule is the paper's: every pair of lattice points closer than
sqrt(3) * spacing is joined (Sec. III-F; the 50^3 lattice of Sec. IV-A has
1,558,396 springs under it).
"""
from __future__ import annotations

import math

import numpy as np

# The 13 "forward" neighbour offsets of the 26-neighbourhood, in
# lexicographic (dz, dy, dx) order; each joins a point to a higher index.
FORWARD_OFFSETS = tuple(
    (dx, dy, dz)
    for dz in (-1, 0, 1)
    for dy in (-1, 0, 1)
    for dx in (-1, 0, 1)
    if (dz, dy, dx) > (0, 0, 0)
)
assert len(FORWARD_OFFSETS) == 13

# Corner offsets of a unit voxel, corner c = bit0 x + bit1 y + bit2 z.
_VOXEL_CORNERS = tuple(((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8))
# All 28 corner pairs of one voxel: 12 edges, 12 face diagonals, 4 body diagonals.
_VOXEL_PAIRS = tuple((a, b) for a in range(8) for b in range(a + 1, 8))
assert len(_VOXEL_PAIRS) == 28


def lattice_spring_count(nx: int, ny: int | None = None, nz: int | None = None) -> int:
    """Number of 26-neighbourhood pairs in an nx*ny*nz point grid (closed form)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    total = 0
    for dx, dy, dz in FORWARD_OFFSETS:
        total += max(nx - abs(dx), 0) * max(ny - abs(dy), 0) * max(nz - abs(dz), 0)
    return total


def lattice_topology(nx: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """Spring end pairs of an nx*ny*nz grid under the 26-neighbourhood rule.

    Point index is ``ix + nx*iy + nx*ny*iz`` (x fastest).  Springs are ordered
    by their lower end, then by the 13 forward offsets in (dz, dy, dx)
    lexicographic order.  Returns an (s, 2) int64 array with ends[:,0] < ends[:,1].
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    ids = np.arange(n, dtype=np.int64)
    ix = ids % nx
    iy = (ids // nx) % ny
    iz = ids // (nx * ny)
    cols = []
    valid = []
    for dx, dy, dz in FORWARD_OFFSETS:
        ok = (
            (ix + dx >= 0) & (ix + dx < nx)
            & (iy + dy >= 0) & (iy + dy < ny)
            & (iz + dz >= 0) & (iz + dz < nz)
        )
        cols.append(ids + dx + nx * dy + nx * ny * dz)
        valid.append(ok)
    other = np.stack(cols, axis=1)  # (n, 13), id-major then offset order
    ok = np.stack(valid, axis=1)
    lo = np.broadcast_to(ids[:, None], other.shape)
    ends = np.stack([lo[ok], other[ok]], axis=1).astype(np.int64)
    return ends


def lattice(
    nx: int,
    ny: int | None = None,
    nz: int | None = None,
    *,
    spacing: float = 0.1,
    origin=(0.0, 0.0, 0.5),
    mass: float = 0.1,
    k: float = 1.0e4,
    damping: float = 1.0,
) -> dict:
    """Unjittered, unactuated cube lattice (no random draws)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    ids = np.arange(n, dtype=np.int64)
    grid = np.stack([ids % nx, (ids // nx) % ny, ids // (nx * ny)], axis=1).astype(np.float64)
    pos = grid * spacing + np.asarray(origin, dtype=np.float64)[None, :]
    ends = lattice_topology(nx, ny, nz)
    s = ends.shape[0]
    return dict(
        pos=pos.astype(np.float32),
        vel=np.zeros((n, 3), np.float32),
        mass=np.full(n, mass, np.float32),
        ends=ends,
        k=np.full(s, k, np.float32),
        damping=np.full(s, damping, np.float32),
        amp=None,
        phase=None,
        body=None,
    )


def cube_drop(n: int = 10) -> dict:
    """Small single cube: n^3 masses, 0.1 m spacing, 0.1 kg, k = 1e4 N/m,
    damping 1 N*s/m, rest length = initial length, lowest layer at z = 0.5 m,
    at rest.  With n = 10 this is the 1,000-mass / 10,476-spring cube."""
    return lattice(n)


def contact_slide(n: int = 10, height: float = 1.0e-3, v0=(0.5, 0.2, 0.0)) -> dict:
    """The small cube placed just above the ground (lowest layer at ``height``)
    and sliding with velocity ``v0``, so that contact and friction act within
    a few hundred steps at dt = 1e-4."""
    sc = lattice(n, origin=(0.0, 0.0, height))
    sc["vel"][:] = np.asarray(v0, np.float32)[None, :]
    return sc


def jittered_actuated_lattice(
    n: int = 100,
    seed: int = 2,
    *,
    spacing: float = 0.1,
    jitter: float = 0.002,
    k_range=(5.0e3, 2.0e4),
    amp: float = 0.1,
    origin=(0.0, 0.0, 0.5),
    mass: float = 0.1,
    damping: float = 1.0,
) -> dict:
    """Large actuated lattice.

    Topology is the n^3 26-neighbourhood grid.  Draws, in this order from
    ``Generator(PCG64(seed))``: position jitter U(-jitter, jitter) per
    coordinate (n^3 x 3), stiffness U(k_range) per spring, phase U(0, 2*pi)
    per spring.  Amplitude is ``amp`` for every spring.  The defaults give the
    1,000,000-mass / 12,731,796-spring lattice (±2% spacing jitter).
    """
    sc = lattice(n, spacing=spacing, origin=origin, mass=mass, damping=damping)
    rng = np.random.Generator(np.random.PCG64(seed))
    npts = sc["pos"].shape[0]
    s = sc["ends"].shape[0]
    jit = rng.uniform(-jitter, jitter, size=(npts, 3))
    kk = rng.uniform(k_range[0], k_range[1], size=s)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=s)
    base = sc["pos"].astype(np.float64)
    sc["pos"] = (base + jit).astype(np.float32)
    sc["k"] = kk.astype(np.float32)
    sc["amp"] = np.full(s, amp, np.float32)
    sc["phase"] = ph.astype(np.float32)
    return sc


# ----------------------------------------------------------------------------
# Voxel robots
# ----------------------------------------------------------------------------

def _largest_component6(occ: np.ndarray) -> np.ndarray:
    """Largest 6-connected (face-sharing) component of a boolean voxel grid.

    Ties go to the component whose first voxel in raster order comes first.
    An empty grid yields an empty mask.
    """
    from scipy import ndimage

    struct = ndimage.generate_binary_structure(3, 1)  # 6-connectivity
    lab, nlab = ndimage.label(occ, structure=struct)
    if nlab == 0:
        return np.zeros_like(occ, dtype=bool)
    sizes = np.bincount(lab.ravel())[1:]
    best = int(np.argmax(sizes)) + 1  # argmax takes the first (lowest label) on ties
    return lab == best


def voxel_robot(rng: np.random.Generator, side_lo: int, side_hi: int, *,
                p_occ: float = 0.6, voxel: float = 0.1, mass: float = 0.1,
                k: float = 1.0e4, damping: float = 1.0, amp_max: float = 0.15) -> dict:
    """One random voxel robot.

    Draws, in order: side ~ U{side_lo..side_hi}; occupancy of all side^3
    voxels ~ Bernoulli(p_occ) (voxel index ix + s*iy + s^2*iz); phase
    U(0, 2*pi) for all side^3 voxels; amplitude U(0, amp_max) for all side^3
    voxels.  The largest 6-connected component is kept (if no voxel is
    occupied, voxel 0 alone is kept).  Masses sit at the distinct corners of
    kept voxels (numbered in corner raster order), springs join every corner
    pair of every kept voxel (edges, face and body diagonals), deduplicated
    and sorted by (lower, upper) mass index.  The lowest corners are at z = 0.

    Each spring's actuation phasor is the mean of ``a*(cos phi, sin phi)`` over
    the kept voxels that contain both its ends; ``amp``/``phase`` are that
    mean's modulus and argument.  ``voxel_a``, ``voxel_phi`` (kept voxels
    only) and the spring->voxel membership (``sv_ptr``, ``sv_idx``) are
    returned so gradients can be mapped back to voxels.
    """
    s = int(rng.integers(side_lo, side_hi + 1))
    occ_flat = rng.random(s ** 3) < p_occ
    phi_all = rng.uniform(0.0, 2.0 * math.pi, size=s ** 3)
    a_all = rng.uniform(0.0, amp_max, size=s ** 3)

    occ = occ_flat.reshape(s, s, s)  # [iz, iy, ix]
    keep = _largest_component6(occ)
    if not keep.any():
        keep = np.zeros_like(occ)
        keep.flat[0] = True
    vflat = np.flatnonzero(keep.ravel())  # kept voxel raster indices
    vx = vflat % s
    vy = (vflat // s) % s
    vz = vflat // (s * s)

    c1 = s + 1
    corner_ids = np.empty((vflat.size, 8), np.int64)
    for c, (ox, oy, oz) in enumerate(_VOXEL_CORNERS):
        corner_ids[:, c] = (vx + ox) + c1 * (vy + oy) + c1 * c1 * (vz + oz)
    used = np.unique(corner_ids)
    remap = np.full(c1 ** 3, -1, np.int64)
    remap[used] = np.arange(used.size)
    mids = remap[corner_ids]  # (nv, 8) mass ids

    # Every corner pair of every voxel, with its voxel.
    pa = np.array([p[0] for p in _VOXEL_PAIRS])
    pb = np.array([p[1] for p in _VOXEL_PAIRS])
    e0 = mids[:, pa].ravel()
    e1 = mids[:, pb].ravel()
    lo = np.minimum(e0, e1)
    hi = np.maximum(e0, e1)
    vox_of_pair = np.repeat(np.arange(vflat.size), len(_VOXEL_PAIRS))
    key = lo * used.size + hi
    order = np.lexsort((vox_of_pair, key))
    key_s = key[order]
    first = np.ones(key_s.size, bool)
    first[1:] = key_s[1:] != key_s[:-1]
    spring_of_pair = np.cumsum(first) - 1
    uniq = order[first]
    ends = np.stack([lo[uniq], hi[uniq]], axis=1)
    nsp = ends.shape[0]
    sv_idx = vox_of_pair[order].astype(np.int32)  # grouped by spring
    sv_ptr = np.zeros(nsp + 1, np.int32)
    np.add.at(sv_ptr, spring_of_pair + 1, 1)
    sv_ptr = np.cumsum(sv_ptr).astype(np.int32)

    ux = used % c1
    uy = (used // c1) % c1
    uz = used // (c1 * c1)
    pos = np.stack([ux, uy, uz - uz.min()], axis=1).astype(np.float64) * voxel

    va = a_all[vflat]
    vphi = phi_all[vflat]
    amp_s, phase_s = voxel_to_spring_actuation(va, vphi, sv_ptr, sv_idx)

    n = used.size
    return dict(
        pos=pos.astype(np.float32),
        vel=np.zeros((n, 3), np.float32),
        mass=np.full(n, mass, np.float32),
        ends=ends.astype(np.int64),
        k=np.full(nsp, k, np.float32),
        damping=np.full(nsp, damping, np.float32),
        amp=amp_s.astype(np.float32),
        phase=phase_s.astype(np.float32),
        body=None,
        side=s,
        voxel_index=vflat.astype(np.int32),
        voxel_a=va,
        voxel_phi=vphi,
        sv_ptr=sv_ptr,
        sv_idx=sv_idx,
    )


def voxel_to_spring_actuation(voxel_a, voxel_phi, sv_ptr, sv_idx):
    """Per-spring (amplitude, phase), FP64, as the polar form of the mean of the
    member voxels' phasors a*(cos phi, sin phi).  This is the scene's
    definition of how voxel actuation drives shared springs."""
    va = np.asarray(voxel_a, np.float64)
    vp = np.asarray(voxel_phi, np.float64)
    cnt = np.diff(sv_ptr).astype(np.float64)
    seg = np.repeat(np.arange(cnt.size), np.diff(sv_ptr))
    c = np.bincount(seg, weights=(va * np.cos(vp))[sv_idx], minlength=cnt.size) / cnt
    s = np.bincount(seg, weights=(va * np.sin(vp))[sv_idx], minlength=cnt.size) / cnt
    return np.hypot(c, s), np.arctan2(s, c)


def robot_batch(count: int, seed: int, side_lo: int, side_hi: int, **kw) -> list[dict]:
    """``count`` robots drawn one after another from ``Generator(PCG64(seed))``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [voxel_robot(rng, side_lo, side_hi, **kw) for _ in range(count)]


def concat(robots: list[dict]) -> dict:
    """Concatenate independent bodies into one scene (``body`` gives the body of
    each mass; ``mass_ptr``/``spring_ptr`` give each body's ranges)."""
    mass_ptr = np.zeros(len(robots) + 1, np.int64)
    spring_ptr = np.zeros(len(robots) + 1, np.int64)
    for b, r in enumerate(robots):
        mass_ptr[b + 1] = mass_ptr[b] + r["pos"].shape[0]
        spring_ptr[b + 1] = spring_ptr[b] + r["ends"].shape[0]
    ends = np.concatenate([r["ends"] + mass_ptr[b] for b, r in enumerate(robots)])

    def cat(key):
        if any(r[key] is None for r in robots):
            return None
        return np.concatenate([r[key] for r in robots])

    body = np.concatenate([np.full(r["pos"].shape[0], b, np.int32) for b, r in enumerate(robots)])
    out = dict(
        pos=cat("pos"), vel=cat("vel"), mass=cat("mass"), ends=ends, k=cat("k"),
        damping=cat("damping"), amp=cat("amp"), phase=cat("phase"), body=body,
        mass_ptr=mass_ptr, spring_ptr=spring_ptr,
    )
    if all("sv_ptr" in r for r in robots):
        # the voxel maps side by side: voxels numbered body after body
        voxel_ptr = np.zeros(len(robots) + 1, np.int64)
        for b, r in enumerate(robots):
            voxel_ptr[b + 1] = voxel_ptr[b] + np.asarray(r["voxel_a"]).size
        sv_ptr = [np.zeros(1, np.int64)]
        base = 0
        for r in robots:
            sv_ptr.append(np.asarray(r["sv_ptr"][1:], np.int64) + base)
            base += int(r["sv_ptr"][-1])
        out.update(
            voxel_a=np.concatenate([r["voxel_a"] for r in robots]),
            voxel_phi=np.concatenate([r["voxel_phi"] for r in robots]),
            voxel_ptr=voxel_ptr,
            sv_ptr=np.concatenate(sv_ptr),
            sv_idx=np.concatenate([np.asarray(r["sv_idx"], np.int64) + voxel_ptr[b]
                                   for b, r in enumerate(robots)]).astype(np.int32),
        )
    return out


# ----------------------------------------------------------------------------
# Worms (wave actuation, Sec. IV-B)
# ----------------------------------------------------------------------------


def worm(nx: int = 27, ny: int = 5, nz: int = 3, *, spacing: float = 0.1, origin=(0.0, 0.0, 0.0),
         mass: float = 0.1, k: float = 1.0e4, damping: float = 1.0, c: float = 0.2) -> dict:
    """A worm: an nx x ny x nz lattice (26-neighbourhood springs, no random
    draws) lying on the ground, long along x, every spring actuated with
    expansion constant ``c`` (the ``amp`` array; ``phase`` is zero).  The
    default 27 x 5 x 3 lattice has 3,392 springs."""
    w = lattice(nx, ny, nz, spacing=spacing, origin=origin, mass=mass, k=k, damping=damping)
    ns = w["ends"].shape[0]
    w["amp"] = np.full(ns, c, np.float32)
    w["phase"] = np.zeros(ns, np.float32)
    return w


def worm_batch(count: int = 100, *, gap: float = 0.3, **kw) -> dict:
    """``count`` identical worms side by side along y, ``gap`` metres apart,
    as independent bodies (100 default worms: 339,200 springs)."""
    ny = kw.get("ny", 5)
    spacing = kw.get("spacing", 0.1)
    x0, y0, z0 = kw.pop("origin", (0.0, 0.0, 0.0))
    step = (ny - 1) * spacing + gap
    return concat([worm(origin=(x0, y0 + q * step, z0), **kw) for q in range(count)])


# ----------------------------------------------------------------------------
# Many small voxel robots at once (surrogate datasets)
# ----------------------------------------------------------------------------

def small_robot_batch(count: int, seed: int, side_lo: int = 3, side_hi: int = 8, *, grid: int = 8,
                      p_occ: float = 0.6, voxel: float = 0.1, mass: float = 0.1, k: float = 1.0e4,
                      damping: float = 1.0, amp_max: float = 0.15) -> dict:
    """``count`` voxel robots of side <= ``grid``, built together.

    Same rules as :func:`voxel_robot` (Bernoulli occupancy, largest
    6-connected component, masses at distinct corners, springs on all 28
    corner pairs of every kept voxel, lowest corners at z = 0, per-spring
    actuation = polar form of the mean voxel phasor), with a bulk draw order
    from ``Generator(PCG64(seed))``: sides (count), then occupancy uniforms,
    phases U(0, 2 pi) and amplitudes U(0, amp_max), each ``count x grid^3``;
    a robot of side s uses the first s^3 values of its row, voxel index
    ix + s*iy + s^2*iz.  Voxels sit at the same (ix, iy, iz) of a
    ``grid^3`` frame, which the returned ``occ``, ``vox_a``, ``vox_phi``
    arrays ([count, grid, grid, grid], index [iz, iy, ix]) describe.

    Returns one concatenated scene (as :func:`concat`) plus those grids.
    """
    from scipy import ndimage

    G = grid
    G3 = G ** 3
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    U = rng.random((count, G3))
    PH = rng.uniform(0.0, 2.0 * math.pi, size=(count, G3))
    AM = rng.uniform(0.0, amp_max, size=(count, G3))

    occ = np.zeros((count, G, G, G), bool)
    vphi = np.zeros((count, G, G, G))
    vamp = np.zeros((count, G, G, G))
    for s in range(side_lo, side_hi + 1):
        rs = np.flatnonzero(sides == s)
        if rs.size == 0:
            continue
        occ[rs, :s, :s, :s] = (U[rs, :s ** 3] < p_occ).reshape(-1, s, s, s)
        vphi[rs, :s, :s, :s] = PH[rs, :s ** 3].reshape(-1, s, s, s)
        vamp[rs, :s, :s, :s] = AM[rs, :s ** 3].reshape(-1, s, s, s)

    # largest face-connected component of every robot in one labelling pass
    struct = np.zeros((3, 3, 3, 3), bool)
    struct[1] = ndimage.generate_binary_structure(3, 1)
    lab, nlab = ndimage.label(occ, structure=struct)
    flat = lab.reshape(count, G3)
    keep = np.zeros((count, G3), bool)
    if nlab:
        sizes = np.bincount(lab.ravel(), minlength=nlab + 1)
        robot_of = np.zeros(nlab + 1, np.int64)
        rr, cc = np.nonzero(flat)
        robot_of[flat[rr, cc]] = rr
        labels = np.arange(1, nlab + 1)
        # per robot: the largest label, ties to the lowest label (raster order)
        order = np.lexsort((labels, -sizes[1:], robot_of[1:]))
        first = np.ones(order.size, bool)
        first[1:] = robot_of[1:][order][1:] != robot_of[1:][order][:-1]
        best = np.zeros(count, np.int64)
        best[robot_of[1:][order][first]] = labels[order][first]
        keep = (flat == best[:, None]) & (flat > 0)
    empty = ~keep.any(axis=1)
    keep[empty, 0] = True
    keep3 = keep.reshape(count, G, G, G)
    occ = keep3
    vphi = np.where(keep3, vphi, 0.0)
    vamp = np.where(keep3, vamp, 0.0)

    # kept voxels: (robot, ix, iy, iz)
    r_v, z_v, y_v, x_v = np.nonzero(keep3)
    nv = r_v.size
    C1 = G + 1
    C3 = C1 ** 3
    corner = np.empty((nv, 8), np.int64)
    for c, (ox, oy, oz) in enumerate(_VOXEL_CORNERS):
        corner[:, c] = r_v * C3 + (x_v + ox) + C1 * (y_v + oy) + C1 * C1 * (z_v + oz)
    used = np.unique(corner)
    mid = np.searchsorted(used, corner)  # global mass index per voxel corner
    pa = np.array([p[0] for p in _VOXEL_PAIRS])
    pb = np.array([p[1] for p in _VOXEL_PAIRS])
    e0 = mid[:, pa].ravel()
    e1 = mid[:, pb].ravel()
    lo = np.minimum(e0, e1)
    hi = np.maximum(e0, e1)
    vox_of_pair = np.repeat(np.arange(nv), len(_VOXEL_PAIRS))
    key = lo * used.size + hi
    order = np.lexsort((vox_of_pair, key))
    key_s = key[order]
    firstk = np.ones(key_s.size, bool)
    firstk[1:] = key_s[1:] != key_s[:-1]
    spring_of_pair = np.cumsum(firstk) - 1
    uniq = order[firstk]
    ends = np.stack([lo[uniq], hi[uniq]], axis=1)
    nsp = ends.shape[0]
    sv_idx = vox_of_pair[order]
    cnt = np.bincount(spring_of_pair, minlength=nsp).astype(np.float64)
    va = vamp[r_v, z_v, y_v, x_v]
    vp = vphi[r_v, z_v, y_v, x_v]
    cs = np.bincount(spring_of_pair, weights=(va * np.cos(vp))[sv_idx], minlength=nsp) / cnt
    sn = np.bincount(spring_of_pair, weights=(va * np.sin(vp))[sv_idx], minlength=nsp) / cnt

    robot = used // C3
    rem = used % C3
    cx, cy, cz = rem % C1, (rem // C1) % C1, rem // (C1 * C1)
    zmin = np.full(count, np.iinfo(np.int64).max)
    np.minimum.at(zmin, robot, cz)
    pos = np.stack([cx, cy, cz - zmin[robot]], axis=1).astype(np.float64) * voxel
    mass_ptr = np.concatenate([[0], np.cumsum(np.bincount(robot, minlength=count))]).astype(np.int64)
    spring_ptr = np.concatenate([[0], np.cumsum(np.bincount(robot[ends[:, 0]], minlength=count))]).astype(np.int64)
    n = used.size
    return dict(
        pos=pos.astype(np.float32), vel=np.zeros((n, 3), np.float32), mass=np.full(n, mass, np.float32),
        ends=ends.astype(np.int64), k=np.full(nsp, k, np.float32), damping=np.full(nsp, damping, np.float32),
        amp=np.hypot(cs, sn).astype(np.float32), phase=np.arctan2(sn, cs).astype(np.float32),
        body=robot.astype(np.int32), mass_ptr=mass_ptr, spring_ptr=spring_ptr, sides=sides,
        occ=occ, vox_a=vamp, vox_phi=vphi,
    )
