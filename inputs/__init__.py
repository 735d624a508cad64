"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module holds random streams and mesh *descriptions* only (grid sizes,
domain extents, stretching factor, point clouds and triangle lists).  It holds
no finite-volume coefficient, operator, solver or layout arithmetic: each side
derives cell volumes, face lengths, distances and matrices on its own.

Random numbers come from one counter-based generator, SplitMix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
value ``i`` of stream ``(seed, stream)`` is ``mix(key + (i + 1) * GAMMA)`` with
``key = mix(seed ^ mix(stream + GAMMA))``.  Uniforms take the top 53 bits;
normals use the Box-Muller transform on consecutive pairs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def u64(seed: int, stream: int, n: int) -> np.ndarray:
    """``n`` raw 64-bit draws of stream ``(seed, stream)``."""
    with np.errstate(over="ignore"):
        key = _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
                   ^ _mix(np.uint64(stream & 0xFFFFFFFFFFFFFFFF) + _GAMMA))
        ctr = np.arange(1, n + 1, dtype=np.uint64) * _GAMMA + key
    return _mix(ctr)


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """Uniform draws on [0, 1) with 53-bit resolution."""
    return (u64(seed, stream, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform(seed: int, stream: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform draws on [lo, hi); the default is U[-1, 1)."""
    return lo + (hi - lo) * uniform01(seed, stream, n)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """Standard normal draws by Box-Muller on pairs of uniforms."""
    m = (n + 1) // 2
    raw = u64(seed, stream, 2 * m) >> np.uint64(11)
    u1 = (raw[0::2].astype(np.float64) + 1.0) * 2.0 ** -53  # (0, 1]
    u2 = raw[1::2].astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * m)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:n]


# --------------------------------------------------------------------------
# Mesh descriptions
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class CartSpec:
    """A 2D structured base mesh, extruded ``k`` times along z.

    x has ``nx`` uniform cells on [x0, x0+Lx]; y has ``ny`` cells on [y0, y1]
    with hyperbolic-tangent clustering of factor ``stretch`` towards both walls
    (``stretch == 0`` means uniform).  ``periodic_x``/``periodic_y`` select
    periodic boundaries; non-periodic boundaries are walls.
    """
    nx: int
    ny: int
    Lx: float
    y0: float
    y1: float
    stretch: float
    periodic_x: bool = True
    periodic_y: bool = False
    x0: float = 0.0

    def as_args(self):
        return (self.nx, self.ny, self.x0, self.Lx, self.y0, self.y1,
                self.stretch, int(self.periodic_x), int(self.periodic_y))


@dataclass(frozen=True)
class TriSpec:
    """A 2D triangle base mesh given as points and vertex triples."""
    points: np.ndarray = field(repr=False)     # (n_pts, 2) float64
    triangles: np.ndarray = field(repr=False)  # (n_tri, 3) int32
    name: str = "tri"


def channel_base(nx: int, ny: int, stretch: float = 1.5) -> CartSpec:
    """Channel-shaped base: x periodic on [0, 2*pi], y walls on [-1, 1]."""
    return CartSpec(nx, ny, 2.0 * math.pi, -1.0, 1.0, stretch, True, False)


def convection_base(nx: int = 160, ny: int = 320, stretch: float = 1.5) -> CartSpec:
    """Convection-cell-shaped base: walls on all four sides, x in [0,1], y in [0,2]."""
    return CartSpec(nx, ny, 1.0, 0.0, 2.0, stretch, False, False)


def naca0012_thickness(x: np.ndarray) -> np.ndarray:
    """Half-thickness of the NACA 0012 section for chord 1, x in [0, 1]."""
    return 0.6 * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                  + 0.2843 * x ** 3 - 0.1015 * x ** 4)


def _inside_naca(px: np.ndarray, py: np.ndarray, margin: float = 0.0) -> np.ndarray:
    """Points inside the section (leading edge at x=-0.5, chord 1, centred at 0)."""
    xc = px + 0.5
    inside = (xc >= 0.0) & (xc <= 1.0)
    t = np.zeros_like(px)
    t[inside] = naca0012_thickness(xc[inside])
    return inside & (np.abs(py) <= t + margin)


def naca_delaunay(seed: int = 1, n_interior: int = 100_000, n_surface: int = 400,
                  n_box_side: int = 100, half_box: float = 10.0,
                  near_fraction: float = 0.5) -> TriSpec:
    """Delaunay mesh around a NACA-0012 section in a 20-chord square box.

    Points: ``n_surface`` cosine-spaced points on the section surface,
    ``n_box_side`` uniform points per box side, and ``n_interior`` random
    points (stream ``(seed, 0..3)``): a fraction ``near_fraction`` drawn with a
    Gaussian cluster around the body, the rest uniform in the box.  Interior
    points inside the body or closer to its surface than the local surface
    spacing are rejected.  Triangles whose centroid lies inside the body are
    dropped.  The triangulation itself is scipy's Qhull Delaunay.
    """
    from scipy.spatial import Delaunay

    m = n_surface // 2
    beta = np.linspace(0.0, math.pi, m + 1)
    xs = 0.5 * (1.0 - np.cos(beta))                     # 0..1 cosine spacing
    yt = naca0012_thickness(xs)
    upper = np.stack([xs - 0.5, yt], axis=1)
    lower = np.stack([xs[1:-1] - 0.5, -yt[1:-1]], axis=1)[::-1]
    surface = np.concatenate([upper, lower[::-1]], axis=0)
    # Trailing edge has finite thickness; keep both trailing points.
    te_low = np.array([[0.5, -yt[-1]]])
    surface = np.concatenate([surface, te_low], axis=0)

    s = np.linspace(-half_box, half_box, n_box_side + 1)
    box = np.concatenate([
        np.stack([s[:-1], np.full(n_box_side, -half_box)], 1),
        np.stack([np.full(n_box_side, half_box), s[:-1]], 1),
        np.stack([s[::-1][:-1], np.full(n_box_side, half_box)], 1),
        np.stack([np.full(n_box_side, -half_box), s[::-1][:-1]], 1),
    ])

    n_near = int(n_interior * near_fraction)
    n_far = n_interior - n_near
    far = np.stack([uniform(seed, 0, n_far, -half_box, half_box),
                    uniform(seed, 1, n_far, -half_box, half_box)], 1)
    g = normal(seed, 2, 2 * n_near).reshape(n_near, 2)
    near = g * np.array([1.0, 0.6])
    near = near[(np.abs(near[:, 0]) < half_box) & (np.abs(near[:, 1]) < half_box)]
    pts = np.concatenate([far, near], axis=0)
    # Keep interior points away from the body by about the surface spacing
    # and away from the box edge by half the box spacing.
    spacing_body = math.pi / m * 0.5
    keep = ~_inside_naca(pts[:, 0], pts[:, 1], margin=spacing_body)
    edge = half_box - 0.5 * (2 * half_box / n_box_side)
    keep &= (np.abs(pts[:, 0]) < edge) & (np.abs(pts[:, 1]) < edge)
    pts = pts[keep]

    allp = np.concatenate([surface, box, pts], axis=0)
    tri = Delaunay(allp).simplices.astype(np.int64)
    cen = allp[tri].mean(axis=1)
    tri = tri[~_inside_naca(cen[:, 0], cen[:, 1])]
    # Drop points no triangle uses, renumber, and orient counter-clockwise.
    used = np.unique(tri)
    remap = -np.ones(len(allp), dtype=np.int64)
    remap[used] = np.arange(len(used))
    tri = remap[tri]
    allp = allp[used]
    a = allp[tri[:, 1]] - allp[tri[:, 0]]
    b = allp[tri[:, 2]] - allp[tri[:, 0]]
    cw = (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]) < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    return TriSpec(np.ascontiguousarray(allp), np.ascontiguousarray(tri.astype(np.int32)),
                   name="naca0012")


def unit_square_triangles(n: int = 3, seed: int = 7, jitter: float = 0.2) -> TriSpec:
    """Tiny jittered Delaunay mesh of the unit square (brute-force tests)."""
    from scipy.spatial import Delaunay
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    p = np.stack([X.ravel(), Y.ravel()], 1)
    interior = (p[:, 0] > 0) & (p[:, 0] < 1) & (p[:, 1] > 0) & (p[:, 1] < 1)
    d = uniform(seed, 0, 2 * len(p), -jitter / n, jitter / n).reshape(-1, 2)
    p[interior] += d[interior]
    tri = Delaunay(p).simplices.astype(np.int64)
    a = p[tri[:, 1]] - p[tri[:, 0]]
    b = p[tri[:, 2]] - p[tri[:, 0]]
    cw = (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]) < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    return TriSpec(p, tri.astype(np.int32), name=f"square{n}")


# --------------------------------------------------------------------------
# Right-hand sides and fields (plane-major: value of cell c on plane l at l*n_b+c)
# --------------------------------------------------------------------------

def rhs_uniform(seed: int, n_total: int, stream: int = 1) -> np.ndarray:
    """U[-1,1) right-hand side, plane-major; zero-mean projection is the solver's job."""
    return uniform(seed, stream, n_total)


@dataclass(frozen=True)
class FourierModes:
    """Parameters of a sum of separable Fourier modes on the channel box.

    The field is ``sum_m a_m cos(kx_m x + px_m) cos(kz_m z + pz_m) cos(n_m pi (y+1)/2)``.
    """
    a: np.ndarray
    kx: np.ndarray
    kz: np.ndarray
    n: np.ndarray
    px: np.ndarray
    pz: np.ndarray

    def evaluate(self, x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
        out = np.zeros(np.broadcast(x, y, z).shape)
        for m in range(len(self.a)):
            out += (self.a[m] * np.cos(self.kx[m] * x + self.px[m])
                    * np.cos(self.kz[m] * z + self.pz[m])
                    * np.cos(self.n[m] * math.pi * (y + 1.0) / 2.0))
        return out

    def advanced(self, omega_x: np.ndarray, omega_z: np.ndarray) -> "FourierModes":
        return FourierModes(self.a, self.kx, self.kz, self.n,
                            self.px + omega_x, self.pz + omega_z)


def fourier_modes(seed: int, stream: int, n_modes: int = 16) -> FourierModes:
    """Random mode set: kx in {0..4}, kz in {0,2,4,6}, n in {0..4}, excluding
    the all-zero triple; amplitudes N(0,1); phases U[0, 2 pi)."""
    raw = u64(seed, stream, 8 * n_modes)
    kx, kz, nn = [], [], []
    i = 0
    while len(kx) < n_modes:
        if i >= len(raw):
            raw = np.concatenate([raw, u64(seed, stream + 1000, 8 * n_modes)])
        a_, b_, c_ = int(raw[i] % 5), 2 * int(raw[i + 1] % 4), int(raw[i + 2] % 5)
        i += 3
        if a_ == 0 and b_ == 0 and c_ == 0:
            continue
        kx.append(a_)
        kz.append(b_)
        nn.append(c_)
    a = normal(seed, stream + 1, n_modes)
    ph = uniform(seed, stream + 2, 2 * n_modes, 0.0, 2.0 * math.pi)
    return FourierModes(a, np.array(kx, float), np.array(kz, float), np.array(nn, float),
                        ph[:n_modes], ph[n_modes:])


# --------------------------------------------------------------------------
# Workload table (sizes of the paper-shaped synthetic cases)
# --------------------------------------------------------------------------

PI = math.pi

SMALL_CHANNEL = dict(base=channel_base(64, 64), k=8, dz=PI / 8)      # 64x64 base, 8 planes
CHANNEL = dict(base=channel_base(192, 128), k=64, dz=PI / 64)         # 192x128 base, 64 planes
CHANNEL_K_SWEEP = (1, 4, 16, 64)
CONVECTION = dict(base=convection_base(160, 320), k=64, dz=PI / 64)  # 160x320 base, 64 planes
AIRFOIL_K = 32
AIRFOIL_DZ = 2.0 / 32


def batch_problems():
    """24 uneven problems: 4 channel bases x 6 plane counts, RHS seed 100+index."""
    bases = [(32, 32), (64, 64), (128, 96), (256, 192)]
    ks = [4, 8, 16, 32, 64, 128]
    out = []
    for bi, (nx, ny) in enumerate(bases):
        for ki, k in enumerate(ks):
            idx = bi * len(ks) + ki
            out.append(dict(base=channel_base(nx, ny), k=k, dz=PI / k, seed=100 + idx))
    return out


# --------------------------------------------------------------------------
# Learned initial guess: training and evaluation data, initial weights
# --------------------------------------------------------------------------

NET_LAYERS = ((2, 32), (32, 32), (32, 32), (32, 1))  # (c_in, c_out) of the 3x3x3 layers


def net_init(seed: int = 6, zero_output_layer: bool = True) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6 / fan_in), fan_in = 27 c_in) and
    zero biases, flat [W[o][c][tap], b[o]] per layer, float32.  The output
    layer starts at zero by default, so that the untrained network returns
    its previous-pressure input."""
    parts = []
    for li, (ci, co) in enumerate(NET_LAYERS):
        bound = math.sqrt(6.0 / (27 * ci))
        w = uniform(seed, 200 + li, co * ci * 27, -bound, bound)
        if zero_output_layer and li == len(NET_LAYERS) - 1:
            w = np.zeros_like(w)
        parts.append(w)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def guess_trajectory(seed: int, traj: int, n_steps: int, n_modes: int = 16,
                     omega_std: float = 0.1) -> list:
    """Mode sets of one trajectory: phases drift by omega ~ N(0, omega_std)
    per mode and step."""
    modes = fourier_modes(seed, 1000 + 10 * traj, n_modes)
    om = omega_std * normal(seed, 1000 + 10 * traj + 5, 2 * n_modes)
    return [modes.advanced(t * om[:n_modes], t * om[n_modes:]) for t in range(n_steps)]


def integrated_rhs(modes: FourierModes, cx: np.ndarray, cy: np.ndarray, area: np.ndarray,
                   k: int, dz: float) -> np.ndarray:
    """Plane-major right-hand side: the mode sum at the cell centres times the
    cell volume (plane l centred at z = (l + 1/2) dz)."""
    z = (np.arange(k) + 0.5) * dz
    f = modes.evaluate(np.asarray(cx)[None, :], np.asarray(cy)[None, :], z[:, None])
    return (f * np.asarray(area)[None, :] * dz).ravel()


def structured_csr(n: int, points: int = 7):
    """CSR arrays (ptr, col, val) of a periodic n x n x n structured matrix
    with 7 (first neighbours along each axis) or 13 (first and second
    neighbours) nonzeros per row and the values of the unit-spacing second
    and fourth-order differences: the square test matrices of the paper's
    Section 2 bounds (n^3 rows)."""
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    i, j, l = idx % n, (idx // n) % n, idx // (n * n)
    offs = [(0, 0, 0)]
    if points == 7:
        w = [-6.0] + [1.0] * 6
        offs += [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    elif points == 13:
        w = [-7.5] + [4.0 / 3.0] * 6 + [-1.0 / 12.0] * 6
        offs += [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        offs += [(2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2)]
    else:
        raise ValueError("points must be 7 or 13")
    cols = np.stack([((i + a) % n) + ((j + b) % n) * n + ((l + c) % n) * n * n for a, b, c in offs], axis=1)
    order = np.argsort(cols, axis=1)
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(np.broadcast_to(np.array(w), cols.shape), order, axis=1)
    ptr = np.arange(N + 1, dtype=np.int64) * len(offs)
    return ptr.astype(np.int32), cols.ravel().astype(np.int32), np.ascontiguousarray(vals.ravel())
