"""Seeded synthetic workloads shaped like the paper's suspensions.

This module only *draws inputs*: body-frame blob layouts, tracking points,
unit quaternions, link/row definitions, forces and multipliers.  It holds none
of the method's arithmetic (no mobility, no constraint Jacobian, no solver).
Orientations are drawn and applied with ``scipy.spatial.transform.Rotation``
so that neither the CPU oracle's rotation matrix nor the GPU kernels are used
to build their own inputs.

Quaternions are stored scalar-first, ``theta = [s, p1, p2, p3]`` as in the
paper's Sec. 2.1; scipy's scalar-last convention is converted here.

Workloads (all lengths in units of the blob radius a = 1, viscosity eta = 1):

* ``filament``   -- one free filament of rigid rods joined by ball joints
  (Sec. 3.2.1 shapes; 20 rods x 4 blobs by default).
* ``ring``       -- a closed loop of rigid bodies joined by ball joints (an
  articulated body with a loop, Sec. 4.2).
* ``blob_filaments``, ``blob_shells`` -- articulated bodies of single-blob
  bodies (Sec. 2.4; the filament and shell arrays of Sec. 3.2), unbounded.
* ``slab``       -- loose blobs above a wall, random sequential addition
  with minimum separation 2a (mobility mat-vec throughput case).
* ``bacteria``   -- spherical-shell heads + rigid helical flagella joined by
  a hinge, above a wall (Sec. 4.4 / 5.2 / 5.3 shapes).
* ``diatoms``    -- stacked rectangular plates with sliding-parallel links
  (Sec. 5.1 shapes), unbounded.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Workload",
    "filament",
    "ring",
    "blob_filaments",
    "blob_shells",
    "slab",
    "bacteria",
    "diatoms",
    "icosphere42",
    "helix80",
    "random_blobs",
    "random_rigid",
    "bacterium_poses",
    "mlp_init_weights",
]


@dataclass
class Workload:
    """Inputs of one constrained-mobility problem (host arrays, float64).

    Blobs of one body are contiguous: body p owns blobs
    ``blob_offset[p]:blob_offset[p+1]``; ``r_ref`` holds them in the body frame.
    Links (point constraints, Eq. constraint): link n joins bodies
    ``pq[n,0]`` (the + end) and ``pq[n,1]`` (the - end, or -1 for a fixed lab
    point), with body-frame arms ``dl_p``, ``dl_q`` and their time derivatives.
    ``nproj[n]`` rows of the link are kept: the rows of ``proj[n, :nproj[n]]``
    (unit vectors in the body frame of the + body) project the link's
    velocity constraint; a plain ball joint keeps all 3 Cartesian rows.
    General rows: ``row_coef[k] = (c_u_p, c_w_p, c_u_q, c_w_q)`` in the body
    frame of body ``row_pq[k,0]``; the row reads c.U = row_rhs[k].
    """

    name: str
    a: float
    eta: float
    wall: bool
    r_ref: np.ndarray          # (N,3)
    blob_offset: np.ndarray    # (M+1,) int32
    q: np.ndarray              # (M,3)
    theta: np.ndarray          # (M,4) scalar-first unit quaternions
    F: np.ndarray              # (M,6) force, torque about q_p
    pq: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    dl_p: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    dl_q: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    dldot_p: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    dldot_q: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    nproj: np.ndarray = field(default_factory=lambda: np.zeros((0,), np.int32))
    proj: np.ndarray = field(default_factory=lambda: np.zeros((0, 3, 3)))
    row_pq: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    row_coef: np.ndarray = field(default_factory=lambda: np.zeros((0, 12)))
    row_rhs: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    body_type: np.ndarray | None = None
    u_slip: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.blob_offset[-1])

    @property
    def M(self) -> int:
        return int(len(self.blob_offset) - 1)

    @property
    def P(self) -> int:
        return int(len(self.pq))

    @property
    def n_rows(self) -> int:
        return int(self.nproj.sum()) + int(len(self.row_rhs))

    @property
    def n_unknowns(self) -> int:
        return 3 * self.N + 6 * self.M + self.n_rows


def _quat_scalar_first(rot: Rotation) -> np.ndarray:
    xyzw = np.atleast_2d(rot.as_quat())
    return np.concatenate([xyzw[:, 3:4], xyzw[:, :3]], axis=1)


def _links(P):
    eye = np.tile(np.eye(3), (P, 1, 1))
    return dict(
        pq=np.zeros((P, 2), np.int32),
        dl_p=np.zeros((P, 3)),
        dl_q=np.zeros((P, 3)),
        dldot_p=np.zeros((P, 3)),
        dldot_q=np.zeros((P, 3)),
        nproj=np.full(P, 3, np.int32),
        proj=eye,
    )


# ---------------------------------------------------------------- filament
def filament(n_rods: int = 20, blobs_per_rod: int = 4, seed: int = 1,
             max_angle: float = 0.3, spacing: float = 2.0) -> Workload:
    """Free filament of collinear-blob rods joined end to end by ball joints.

    Rod p has blobs at body-frame x in {-3,-1,1,3} (spacing 2a); joint n sits
    at +4 e_x of rod n and -4 e_x of rod n+1 (the filament link of Sec. 3.2.1
    with l_c = 8a).  Joint angles are drawn U(-max_angle, max_angle) as
    rotations about the lab y axis (a planar bend), and rod centres are laid
    out by walking the chain so that every joint coincides at t = 0.
    Forces and torques are N(0,1); the torque component along each rod axis
    is removed, because collinear blobs give that spin no hydrodynamic
    resistance (the system is consistent only without it).
    """
    rng = np.random.default_rng(seed)
    half = 0.5 * spacing * blobs_per_rod
    xs = (np.arange(blobs_per_rod) - 0.5 * (blobs_per_rod - 1)) * spacing
    r_ref = np.zeros((n_rods * blobs_per_rod, 3))
    r_ref[:, 0] = np.tile(xs, n_rods)
    blob_offset = np.arange(n_rods + 1, dtype=np.int32) * blobs_per_rod
    alpha = rng.uniform(-max_angle, max_angle, n_rods - 1)
    beta = np.concatenate([[0.0], np.cumsum(alpha)])
    theta = np.stack([np.cos(beta / 2), 0 * beta, np.sin(beta / 2), 0 * beta], 1)
    axis = np.stack([np.cos(beta), 0 * beta, -np.sin(beta)], 1)   # rod direction
    q = np.zeros((n_rods, 3))
    for p in range(n_rods - 1):
        q[p + 1] = q[p] + half * axis[p] + half * axis[p + 1]
    F = rng.standard_normal((n_rods, 6))
    tau_ax = np.einsum("ij,ij->i", F[:, 3:], axis)
    F[:, 3:] -= tau_ax[:, None] * axis
    L = _links(n_rods - 1)
    for n in range(n_rods - 1):
        L["pq"][n] = (n, n + 1)
        L["dl_p"][n] = (half, 0, 0)
        L["dl_q"][n] = (-half, 0, 0)
    return Workload("filament", 1.0, 1.0, False, r_ref, blob_offset, q, theta, F,
                    extra=dict(axis=axis, beta=beta), **L)


# ---------------------------------------------------------------- ring
def ring(n_bodies: int = 8, seed: int = 8, wall: bool = False, height: float = 12.0,
         tilt: float = 0.0) -> Workload:
    """Closed loop of rigid bodies joined end to end by ball joints.

    Each body has blobs at body-frame (x, 0, 0), x in {-3,-1,1,3}, plus one at
    (0, 0, 1.8), so that it resists every rotation (no spin null space).
    Joint n sits at +4 e_x of body n and -4 e_x of body n+1 (mod n_bodies); at
    t = 0 the joints are the vertices of a regular polygon of side 8 in the
    plane z = height (tilted by ``tilt`` radians about the lab x axis), so
    every link holds.  Forces and torques are N(0,1) per body.  With
    ``wall`` the no-slip wall z = 0 is present.
    """
    rng = np.random.default_rng(seed)
    r_body = np.array([[-3.0, 0, 0], [-1.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0], [0, 0, 1.8]])
    Rc = 4.0 / np.sin(np.pi / n_bodies)
    ang = 2 * np.pi * np.arange(n_bodies + 1) / n_bodies
    V = np.stack([Rc * np.cos(ang), Rc * np.sin(ang), 0 * ang], 1)
    tilt_rot = Rotation.from_rotvec([tilt, 0, 0])
    q = np.zeros((n_bodies, 3))
    theta = np.zeros((n_bodies, 4))
    for p in range(n_bodies):
        d = V[p + 1] - V[p]
        rot = tilt_rot * Rotation.from_rotvec([0, 0, np.arctan2(d[1], d[0])])
        q[p] = tilt_rot.apply(0.5 * (V[p] + V[p + 1])) + np.array([0, 0, height])
        theta[p] = _quat_scalar_first(rot)[0]
    r_ref = np.tile(r_body, (n_bodies, 1))
    blob_offset = np.arange(n_bodies + 1, dtype=np.int32) * len(r_body)
    F = rng.standard_normal((n_bodies, 6))
    L = _links(n_bodies)
    for n in range(n_bodies):
        L["pq"][n] = (n, (n + 1) % n_bodies)
        L["dl_p"][n] = (4.0, 0, 0)
        L["dl_q"][n] = (-4.0, 0, 0)
    return Workload("ring", 1.0, 1.0, wall, r_ref, blob_offset, q, theta, F, **L)


# ---------------------------------------------------------------- blobs
def _rsa(rng, n, lo, hi, dmin, existing=None, max_tries=200):
    """Random sequential addition of points in a box with minimum distance."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    cell = dmin
    grid: dict = {}
    pts = []

    def ok(p):
        c = tuple((p // cell).astype(int))
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for k in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        if np.sum((pts[k] - p) ** 2) < dmin * dmin:
                            return False
        return True

    while len(pts) < n:
        for _ in range(max_tries):
            p = lo + (hi - lo) * rng.random(3)
            if ok(p):
                break
        else:
            raise RuntimeError("random sequential addition jammed")
        grid.setdefault(tuple((p // cell).astype(int)), []).append(len(pts))
        pts.append(p)
    return np.array(pts)


def slab(n: int = 16384, side: float = 400.0, zlo: float = 1.5, zhi: float = 20.0,
         dmin: float = 2.0, seed: int = 2) -> dict:
    """Loose blobs in [0,side)^2 x [zlo,zhi] above the wall, min separation dmin.

    Returns ``dict(pos=(n,3), lam=(n,3), a, eta)``; lam ~ N(0,1) per component.
    """
    rng = np.random.default_rng(seed)
    pos = _rsa(rng, n, (0, 0, zlo), (side, side, zhi), dmin)
    lam = rng.standard_normal((n, 3))
    return dict(pos=pos, lam=lam, a=1.0, eta=1.0)


def loose_blobs(pos, a: float = 1.0, eta: float = 1.0, wall: bool = True,
                name: str = "loose blobs") -> Workload:
    """Loose blobs as a workload: every blob a body of one blob at its tracking
    point (identity orientation, no links, zero forces), so that a context holds
    their positions as its state."""
    pos = np.asarray(pos, float).reshape(-1, 3)
    n = len(pos)
    theta = np.zeros((n, 4))
    theta[:, 0] = 1.0
    return Workload(name, a, eta, wall, np.zeros((n, 3)), np.arange(n + 1, dtype=np.int32),
                    pos.copy(), theta, np.zeros((n, 6)), **_links(0))


def random_blobs(n: int, seed: int, box: float = 8.0, zlo: float = 1.2,
                 zhi: float = 6.0, overlap: bool = True) -> dict:
    """Small random blob clouds for parity tests (overlaps allowed)."""
    rng = np.random.default_rng(seed)
    if overlap:
        pos = np.column_stack([rng.uniform(0, box, n), rng.uniform(0, box, n),
                               rng.uniform(zlo, zhi, n)])
    else:
        pos = _rsa(rng, n, (0, 0, zlo), (box, box, zhi), 2.0)
    lam = rng.standard_normal((n, 3))
    return dict(pos=pos, lam=lam, a=1.0, eta=1.0)


# ---------------------------------------------------------------- bacteria
def _icosahedron():
    """Unit icosahedron vertices (12,3) and its 30 edges (i < j, in scan order)."""
    t = (1 + 5 ** 0.5) / 2
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    v /= np.linalg.norm(v, axis=1)[:, None]
    d = np.linalg.norm(v[:, None] - v[None], axis=2)
    emin = d[d > 1e-9].min()
    edges = [(i, j) for i in range(12) for j in range(i + 1, 12) if abs(d[i, j] - emin) < 1e-9]
    assert len(edges) == 30
    return v, edges


def icosphere42(radius: float = 5.0) -> np.ndarray:
    """12 icosahedron vertices + 30 edge midpoints pushed to the sphere."""
    v, edges = _icosahedron()
    mids = [(v[i] + v[j]) / np.linalg.norm(v[i] + v[j]) for i, j in edges]
    pts = np.vstack([v, np.array(mids)])
    assert pts.shape == (42, 3)
    return radius * pts


# ---------------------------------------------------------------- single-blob bodies
def _single_blob_links(x, theta, pairs):
    """Ball joints midway between blob centres x[p], x[q] for every (p, q) pair,
    arms expressed in each body's frame (rotation theta, scalar first)."""
    rot = Rotation.from_quat(np.concatenate([theta[:, 1:], theta[:, :1]], axis=1))
    L = _links(len(pairs))
    for n, (p, qq) in enumerate(pairs):
        mid = 0.5 * (x[p] + x[qq])
        L["pq"][n] = (p, qq)
        L["dl_p"][n] = rot[p].inv().apply(mid - x[p])
        L["dl_q"][n] = rot[qq].inv().apply(mid - x[qq])
    return L


def blob_filaments(nx: int = 1, nz: int = 1, n_blobs: int = 15, lc: float = 2.5,
                   gap: float = 4.0, seed: int = 31) -> Workload:
    """Array of straight filaments of single-blob bodies along x (Sec. 3.2.1).

    Each filament has n_blobs bodies spaced lc apart, joined by ball joints
    midway (dl = +-lc/2 e_x); filaments sit on an nx x nz grid in the (x, z)
    plane with surface gaps of ``gap`` end to end along x and side by side
    along z (centre lines gap + 2a apart; local area fraction about 0.3).
    Every body carries the force (0, 0, -1) (gravity along -z) and no torque.
    Unbounded; the blobs sit at the tracking points.
    """
    length = (n_blobs - 1) * lc + 2.0
    q, pairs = [], []
    for iz in range(nz):
        for ix in range(nx):
            b0 = len(q)
            for k in range(n_blobs):
                q.append([ix * (length + gap) + k * lc, 0.0, iz * (gap + 2.0)])
            pairs += [(b0 + k, b0 + k + 1) for k in range(n_blobs - 1)]
    q = np.array(q, float)
    M = len(q)
    theta = np.tile([1.0, 0, 0, 0], (M, 1))
    F = np.zeros((M, 6))
    F[:, 2] = -1.0
    return Workload("blob_filaments", 1.0, 1.0, False, np.zeros((M, 3)),
                    np.arange(M + 1, dtype=np.int32), q, theta, F,
                    extra=dict(single_blob=True), **_single_blob_links(q, theta, pairs))


def _shell_mesh(level: int):
    """Unit-sphere shell points and links after `level` subdivisions of the
    icosahedron (12, 42, 162, 642 points for 0..3): each subdivision adds the
    projected midpoint of every edge and splits every face in four; the links
    join each point of the last subdivision to the two ends of its edge (60,
    240, 960 for levels 1..3).  Level 1 is the 42-point shell with its points
    and links in the icosahedron's edge order."""
    v, edges = _icosahedron()
    es = set(edges)
    faces = [(i, j, k) for (i, j) in edges for k in range(j + 1, 12)
             if (i, k) in es and (j, k) in es]
    pts = [p for p in v]
    links = []
    for _ in range(level):
        mid = {}
        for (i, j) in edges:
            mid[(i, j)] = len(pts)
            m = pts[i] + pts[j]
            pts.append(m / np.linalg.norm(m))
        links = [(i, mid[(i, j)]) for (i, j) in edges] + [(j, mid[(i, j)]) for (i, j) in edges]
        e = lambda a, b: mid[(min(a, b), max(a, b))]
        faces = [f for (a, b, c) in faces for f in ((a, e(a, b), e(c, a)), (b, e(b, c), e(a, b)),
                                                    (c, e(c, a), e(b, c)),
                                                    (e(a, b), e(b, c), e(c, a)))]
        edges = sorted({(min(x, y), max(x, y)) for f in faces for x, y in
                        ((f[0], f[1]), (f[1], f[2]), (f[2], f[0]))})
    return np.array(pts), links


def blob_shells(n_side: int = 1, lc: float = 2.5, forcing: str = "random",
                seed: int = 32, centres=None, level: int = 1) -> Workload:
    """Cubic lattice of n_side^3 deformable shells of single-blob bodies (Sec. 3.2.2);
    with ``centres`` ((k, 3), in units of the shell radius R) the shells sit there
    instead (the two sedimenting shells of Sec. 4.4 at (+-1.5, 0, +-1.5) R); ``level``
    2 or 3 gives the 162- and 642-point shells of Sec. 4.4 (240 and 960 links).

    A shell is the 42-point icosphere (12 icosahedron vertices, 30 projected
    edge midpoints) scaled so that a vertex and a neighbouring midpoint are lc
    apart; each midpoint is linked to the two vertices of its edge (60 links:
    the midpoints have 2 neighbours, the vertices 5).  Shell centres are two
    diameters apart.  Bodies get random orientations (the link arms follow);
    ``forcing`` = "random": N(0,1) forces and torques, "gravity": (0, 0, -1).
    Unbounded.
    """
    rng = np.random.default_rng(seed)
    unit, pairs1 = _shell_mesh(level)
    R = lc / np.linalg.norm(unit[pairs1[0][0]] - unit[pairs1[0][1]])
    shell = R * unit
    q, pairs = [], []
    if centres is None:
        centres = [4.0 * np.array([ix, iy, iz], float) for ix in range(n_side)
                   for iy in range(n_side) for iz in range(n_side)]
    for c in np.asarray(centres, float).reshape(-1, 3):
        b0 = len(q)
        q.extend(shell + R * c)
        pairs += [(b0 + a, b0 + b) for a, b in pairs1]
    q = np.array(q)
    M = len(q)
    theta = _quat_scalar_first(Rotation.random(M, random_state=rng))
    if forcing == "random":
        F = rng.standard_normal((M, 6))
    else:
        F = np.zeros((M, 6))
        F[:, 2] = -1.0
    return Workload("blob_shells", 1.0, 1.0, False, np.zeros((M, 3)),
                    np.arange(M + 1, dtype=np.int32), q, theta, F,
                    extra=dict(single_blob=True, shell_radius=R),
                    **_single_blob_links(q, theta, pairs))


def helix80(n: int = 80, length: float = 40.0, pitch: float = 10.0,
            radius: float = 2.0) -> np.ndarray:
    """Constant-radius helix (radius cos(2 pi z/pitch), radius sin(...), z)."""
    z = length * np.arange(n) / (n - 1)
    return np.column_stack([radius * np.cos(2 * np.pi * z / pitch),
                            radius * np.sin(2 * np.pi * z / pitch), z])


def bacteria(n_bact: int = 1024, side: float | None = None, seed: int = 3,
             hmin: float = 8.0, hmax: float = 15.0, zmin: float = 1.5,
             literal_hinge: bool = False, head_radius: float = 5.0,
             n_flag: int = 80, motor_rate: float = 1.0) -> Workload:
    """Bacteria above a wall: 42-blob shell head + 80-blob helical flagellum.

    Hinge (Sec. 4.4): link 1 joins head (0,0,R+a) to flagellum (0,0,-a); link 2
    joins head (0,0,2R+a) to flagellum (0,0,R-a).  Default rows: link 1 whole
    (3 rows), link 2 projected on the head-frame x and y axes (2 rows, the
    component along the axis repeats link 1), and one motor row
    (w_flag - w_head) . e_axis = motor_rate.  ``literal_hinge`` keeps all 6
    link rows plus the motor row (rank 6 of 7).
    Head centres: uniform in [0, side)^2 x [hmin, hmax]; orientation uniform,
    redrawn until every blob has z >= zmin and lies >= 2a from the blobs of
    bacteria already placed.  The flagellum frame is the head frame turned
    about the shared axis by a U[0, 2 pi) phase.
    """
    rng = np.random.default_rng(seed)
    a = 1.0
    R = head_radius
    if side is None:
        side = 96.0 * math.sqrt(n_bact)
    head = icosphere42(R)
    flag = helix80(n_flag)
    f_origin = np.array([0.0, 0.0, R + 2 * a])        # flagellum origin, head frame
    nh, nf = len(head), len(flag)
    M = 2 * n_bact
    r_ref = np.vstack([np.vstack([head, flag]) for _ in range(n_bact)])
    sizes = np.tile([nh, nf], n_bact)
    blob_offset = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    q = np.zeros((M, 3))
    theta = np.zeros((M, 4))
    cell = 2.0
    grid: dict = {}
    placed = []

    def clash(pts):
        for p in pts:
            c = (p // cell).astype(int)
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for k in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                            if np.sum((placed[k] - p) ** 2) < 4.0 * a * a:
                                return True
        return False

    for b in range(n_bact):
        for _ in range(100000):
            centre = np.array([rng.uniform(0, side), rng.uniform(0, side),
                               rng.uniform(hmin, hmax)])
            rot_h = Rotation.random(random_state=rng)
            phase = rng.uniform(0, 2 * np.pi)
            rot_f = rot_h * Rotation.from_rotvec([0.0, 0.0, phase])
            fq = centre + rot_h.apply(f_origin)
            pts = np.vstack([centre + rot_h.apply(head), fq + rot_f.apply(flag)])
            if pts[:, 2].min() < zmin:
                continue
            if clash(pts):
                continue
            break
        else:
            raise RuntimeError("could not place bacterium")
        for p in pts:
            grid.setdefault(tuple((p // cell).astype(int)), []).append(len(placed))
            placed.append(p)
        q[2 * b] = centre
        q[2 * b + 1] = fq
        theta[2 * b] = _quat_scalar_first(rot_h)[0]
        theta[2 * b + 1] = _quat_scalar_first(rot_f)[0]
    F = np.zeros((M, 6))
    P = 2 * n_bact
    L = _links(P)
    rows_pq, rows_coef, rows_rhs = [], [], []
    for b in range(n_bact):
        h, f = 2 * b, 2 * b + 1
        n1, n2 = 2 * b, 2 * b + 1
        L["pq"][n1] = (h, f)
        L["dl_p"][n1] = (0, 0, R + a)
        L["dl_q"][n1] = (0, 0, -a)
        L["pq"][n2] = (h, f)
        L["dl_p"][n2] = (0, 0, 2 * R + a)
        L["dl_q"][n2] = (0, 0, R - a)
        if not literal_hinge:
            L["nproj"][n2] = 2
            L["proj"][n2] = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 0]])
        rows_pq.append((h, f))
        rows_coef.append([0, 0, 0, 0, 0, -1.0, 0, 0, 0, 0, 0, 1.0])
        rows_rhs.append(motor_rate)
    body_type = np.tile(np.array([0, 1], np.int32), n_bact)
    return Workload("bacteria", a, 1.0, True, r_ref, blob_offset, q, theta, F,
                    row_pq=np.array(rows_pq, np.int32).reshape(-1, 2),
                    row_coef=np.array(rows_coef, float).reshape(-1, 12),
                    row_rhs=np.array(rows_rhs, float),
                    body_type=body_type, extra=dict(side=side), **L)


# ---------------------------------------------------------------- diatoms
def diatoms(n_col: int = 256, kmin: int = 5, kmax: int = 40, seed: int = 4,
            nx: int = 15, ny: int = 3, spacing: float = 0.81, gap: float = 2.0,
            freq: float = 1.0, dphi: float = 2 * np.pi / 10, t: float = 0.0,
            lattice=(8, 8, 4), literal: bool = False) -> Workload:
    """Colonies of stacked plates with sliding-parallel links (Sec. 5.1).

    Plate = nx x ny blobs in its body xy-plane at the given spacing; plates of
    a colony stack along body z at ``gap``.  Between plates p and p+1 (pair n):
    link 1: dl_p = L/2 e_x + (gap/2) e_z, dl_q = -dl_p; link 2: dl_p =
    L e_x + gap e_z, dl_q = 0, with L = A sin(2 pi f t + (n-1) dphi) and
    A = half the plate length.  Link 2 keeps the 2 rows normal to the segment
    joining the two joints (its 3rd row repeats link 1) unless ``literal``.
    Colonies sit on a lattice of spacing (largest bounding box + 10a), each
    with a random yaw.  Unbounded domain.
    """
    rng = np.random.default_rng(seed)
    a = 1.0
    xs = (np.arange(nx) - 0.5 * (nx - 1)) * spacing
    ys = (np.arange(ny) - 0.5 * (ny - 1)) * spacing
    plate = np.array([[x, y, 0.0] for y in ys for x in xs])
    Lp = (nx - 1) * spacing
    A = 0.5 * Lp
    ks = rng.integers(kmin, kmax + 1, n_col)
    colonies = []
    for K in ks:
        phi = np.arange(K - 1) * dphi
        Ls = A * np.sin(2 * np.pi * freq * t + phi)
        Ld = 2 * np.pi * freq * A * np.cos(2 * np.pi * freq * t + phi)
        centres = np.zeros((K, 3))
        for n in range(K - 1):
            centres[n + 1] = centres[n] + np.array([Ls[n], 0.0, gap])
        centres -= centres.mean(0)
        colonies.append((K, centres, Ls, Ld))
    ext = max(np.ptp(c[:, 0]) + Lp for _, c, _, _ in colonies)
    ext = max(ext, max(np.ptp(c[:, 2]) for _, c, _, _ in colonies) + 2)
    spacing_lat = ext + 10.0
    sites = [(i, j, k) for i in range(lattice[0]) for j in range(lattice[1])
             for k in range(lattice[2])]
    assert len(sites) >= n_col
    r_ref, q, theta, sizes = [], [], [], []
    L = {k: [] for k in ("pq", "dl_p", "dl_q", "dldot_p", "dldot_q", "nproj", "proj")}
    body = 0
    for c, (K, centres, Ls, Ld) in enumerate(colonies):
        yaw = rng.uniform(0, 2 * np.pi)
        rot = Rotation.from_rotvec([0, 0, yaw])
        origin = np.array(sites[c], float) * spacing_lat
        quat = _quat_scalar_first(rot)[0]
        for k in range(K):
            r_ref.append(plate)
            sizes.append(len(plate))
            q.append(origin + rot.apply(centres[k]))
            theta.append(quat)
        for n in range(K - 1):
            p, qq = body + n, body + n + 1
            d1 = np.array([0.5 * Ls[n], 0, 0.5 * gap])
            d2 = np.array([Ls[n], 0, gap])
            seg = d2 - d1
            nrm = np.array([-seg[2], 0.0, seg[0]]) / np.hypot(seg[0], seg[2])
            for (dp, dq, dpd, dqd, proj2) in (
                (d1, -d1, np.array([0.5 * Ld[n], 0, 0]), np.array([-0.5 * Ld[n], 0, 0]), False),
                (d2, np.zeros(3), np.array([Ld[n], 0, 0]), np.zeros(3), True),
            ):
                L["pq"].append((p, qq))
                L["dl_p"].append(dp)
                L["dl_q"].append(dq)
                L["dldot_p"].append(dpd)
                L["dldot_q"].append(dqd)
                if proj2 and not literal:
                    L["nproj"].append(2)
                    L["proj"].append(np.array([[0, 1.0, 0], nrm, [0, 0, 0]]))
                else:
                    L["nproj"].append(3)
                    L["proj"].append(np.eye(3))
        body += K
    M = body
    blob_offset = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    F = np.zeros((M, 6))
    return Workload("diatoms", a, 1.0, False, np.vstack(r_ref), blob_offset,
                    np.array(q), np.array(theta), F,
                    pq=np.array(L["pq"], np.int32), dl_p=np.array(L["dl_p"]),
                    dl_q=np.array(L["dl_q"]), dldot_p=np.array(L["dldot_p"]),
                    dldot_q=np.array(L["dldot_q"]),
                    nproj=np.array(L["nproj"], np.int32), proj=np.array(L["proj"]),
                    extra=dict(plates=ks))


# ---------------------------------------------------------------- small rigid
def random_rigid(n_bodies: int = 3, blobs: int = 12, seed: int = 7,
                 wall: bool = True, links: str = "chain") -> Workload:
    """Tiny articulated assemblies for CPU/GPU parity: icosahedral 12-blob
    spheres (radius 2a) in a chain joined by ball joints at the contact
    points, random orientations, N(0,1) forces/torques and slip."""
    rng = np.random.default_rng(seed)
    ico = icosphere42(2.0)[:blobs]
    r_ref = np.vstack([ico] * n_bodies)
    blob_offset = (np.arange(n_bodies + 1) * blobs).astype(np.int32)
    q = np.zeros((n_bodies, 3))
    rots = Rotation.random(n_bodies, random_state=rng)
    theta = _quat_scalar_first(rots)
    q[:, 0] = 5.0 * np.arange(n_bodies)
    q[:, 2] = 6.0
    F = rng.standard_normal((n_bodies, 6))
    nl = n_bodies - 1 if links == "chain" else 0
    L = _links(nl)
    for n in range(nl):
        # joint midway between consecutive centres, expressed in each body frame
        mid = 0.5 * (q[n] + q[n + 1])
        L["pq"][n] = (n, n + 1)
        L["dl_p"][n] = rots[n].inv().apply(mid - q[n])
        L["dl_q"][n] = rots[n + 1].inv().apply(mid - q[n + 1])
    u_slip = rng.standard_normal((n_bodies * blobs, 3))
    return Workload("rigid", 1.0, 1.0, wall, r_ref, blob_offset, q, theta, F,
                    u_slip=u_slip, **L)


# ---------------------------------------------------------------- learned mobility
def bacterium_poses(n_bact: int, seed: int = 5, hmin: float = 8.0, hmax: float = 15.0,
                    zmin: float = 1.5, head_radius: float = 5.0, n_flag: int = 80):
    """Independent single-bacterium poses above the wall for training data.

    Same geometry and height/orientation law as ``bacteria`` but without mutual
    placement: every head centre sits at x = y = 0 (the wall is invariant under
    in-plane shifts and the per-body mobility ignores other bodies).  Returns a
    Workload with 2 bodies per bacterium (head type 0, flagellum type 1), no
    constraints."""
    rng = np.random.default_rng(seed)
    a = 1.0
    R = head_radius
    head = icosphere42(R)
    flag = helix80(n_flag)
    f_origin = np.array([0.0, 0.0, R + 2 * a])
    qs, ths = [], []
    todo = n_bact
    while todo > 0:
        m = max(2 * todo, 64)
        h = rng.uniform(hmin, hmax, m)
        rot_h = Rotation.random(m, random_state=rng)
        phase = rng.uniform(0, 2 * np.pi, m)
        rot_f = rot_h * Rotation.from_rotvec(np.column_stack([0 * phase, 0 * phase, phase]))
        centre = np.column_stack([0 * h, 0 * h, h])
        fq = centre + rot_h.apply(f_origin)
        zh = np.min(centre[:, None, 2] + np.einsum("mij,kj->mki", rot_h.as_matrix(), head)[..., 2], 1)
        zf = np.min(fq[:, None, 2] + np.einsum("mij,kj->mki", rot_f.as_matrix(), flag)[..., 2], 1)
        ok = np.where((zh >= zmin) & (zf >= zmin))[0][:todo]
        for k in ok:
            qs += [centre[k], fq[k]]
            ths += [_quat_scalar_first(rot_h[int(k)])[0], _quat_scalar_first(rot_f[int(k)])[0]]
        todo -= len(ok)
    M = 2 * n_bact
    r_ref = np.vstack([np.vstack([head, flag]) for _ in range(n_bact)])
    sizes = np.tile([len(head), len(flag)], n_bact)
    blob_offset = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return Workload("bacterium_poses", a, 1.0, True, r_ref, blob_offset, np.array(qs),
                    np.array(ths), np.zeros((M, 6)),
                    body_type=np.tile(np.array([0, 1], np.int32), n_bact))


def mlp_init_weights(seed: int = 6, sizes=(7, 128, 128, 21)) -> np.ndarray:
    """He-normal initial weights (zero biases) of the body-mobility network, flat
    in layer order [W1 (out x in), b1, W2, b2, W3, b3], float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        nin, nout = sizes[i], sizes[i + 1]
        parts.append((rng.standard_normal((nout, nin)) * np.sqrt(2.0 / nin)).ravel())
        parts.append(np.zeros(nout))
    return np.concatenate(parts).astype(np.float32)
