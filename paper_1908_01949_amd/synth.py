"""Seeded synthetic inputs for the seed scan: detector geometry, field maps and events.

This module is a small detector simulation. It produces the *inputs* of the seed
scan (wire table, field map, per-event hits and the truth seed of each track) and
holds none of the scan's own arithmetic: no Runge-Kutta-Nystrom stepping, no
chord/wire distance, no score. Truth tracks are traced with the exact helix in a
uniform field and with a classical fourth-order Runge-Kutta integration of the
first-order system (x, T) on a fine analytic-solenoid table otherwise; the true
distance of a wire to the track is found by dense sampling of the continuous
trajectory followed by a golden-section refinement on its cubic Hermite
interpolant. Both the GPU library and the CPU oracle read what this module
produces and nothing else of it.

Units: mm, MeV/c, tesla, elementary charge. Electrons have q = -1.

Setting (paper, section 1 and 2.1): an electron from a stopping target near the
axis, a 1 T solenoid, a drift chamber with 18 stereo sense layers, and the seed
defined on the cylinder R0 = 500 mm in front of the first layer.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable

import numpy as np

KAPPA = 0.299792458          # (MeV/c) per (T mm e): 1/R[mm] = KAPPA * B[T] / pT[MeV/c]
R0_SEED = 500.0              # seed cylinder radius, mm (section 2.1)
P_SIGNAL = 104.97            # signal electron momentum, MeV/c (section 1)
ELECTRON_Q = -1.0
BASE_SEED = 190801949        # root of every numpy SeedSequence used here


# --------------------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Geometry:
    """Finite straight stereo sense wires; wire i is the segment m_i +- half_len_i * u_i."""
    mx: np.ndarray
    my: np.ndarray
    mz: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    half_len: np.ndarray
    layer_of: np.ndarray          # int32
    layer_rmin: np.ndarray        # radial extent of each layer's wires (waist), mm
    layer_rmax: np.ndarray        # radial extent at the end plates (stereo bulge), mm
    layer_radius: np.ndarray      # waist radius r_l
    layer_nwires: np.ndarray      # int32
    layer_first: np.ndarray       # int32, global id of wire 0 of each layer
    layer_stereo: np.ndarray      # stereo angle (rad)
    half_z: float

    @property
    def n_wires(self) -> int:
        return int(self.mx.shape[0])

    @property
    def n_layers(self) -> int:
        return int(self.layer_rmin.shape[0])


def make_geometry(n_layers: int = 18, r_first: float = 530.0, r_last: float = 820.0,
                  n0: int = 200, dn: int = 10, stereo: float = 0.070,
                  half_z: float = 750.0) -> Geometry:
    """18 layers at radii 530..820 mm, 200+10*l wires, stereo +-70 mrad alternating, |z| <= 750.

    The layer radius is read as the waist (z = 0) radius; the end-plate radius is
    sqrt(r^2 + (half_z tan alpha)^2). Odd layers are staggered by half a cell.
    """
    mx, my, mz, ux, uy, uz, hl, lo = ([] for _ in range(8))
    radius, nwires, first, rmin, rmax, alpha_l = [], [], [], [], [], []
    g = 0
    for l in range(n_layers):
        r = r_first + (r_last - r_first) * l / (n_layers - 1)
        n = n0 + dn * l
        a = stereo if l % 2 == 0 else -stereo
        phi = 2.0 * np.pi * (np.arange(n) + 0.5 * (l % 2)) / n
        mx.append(r * np.cos(phi)); my.append(r * np.sin(phi)); mz.append(np.zeros(n))
        ux.append(-math.sin(a) * np.sin(phi)); uy.append(math.sin(a) * np.cos(phi))
        uz.append(np.full(n, math.cos(a)))
        hl.append(np.full(n, half_z / math.cos(a)))
        lo.append(np.full(n, l, dtype=np.int32))
        radius.append(r); nwires.append(n); first.append(g); alpha_l.append(a)
        rmin.append(r); rmax.append(math.sqrt(r * r + (half_z * math.tan(a)) ** 2))
        g += n
    cat = np.concatenate
    return Geometry(cat(mx), cat(my), cat(mz), cat(ux), cat(uy), cat(uz), cat(hl),
                    cat(lo).astype(np.int32), np.array(rmin), np.array(rmax),
                    np.array(radius), np.array(nwires, dtype=np.int32),
                    np.array(first, dtype=np.int32), np.array(alpha_l), half_z)


# --------------------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Field:
    """Either uniform (bz set, grid None) or an (r, z) grid of (B_r, B_z), [nz][nr] row-major."""
    kind: str                      # "uniform" | "rz"
    bz: float = 1.0
    nr: int = 0
    nz: int = 0
    r0: float = 0.0
    r1: float = 0.0
    z0: float = 0.0
    z1: float = 0.0
    br_grid: np.ndarray | None = None   # float32 [nz][nr]
    bz_grid: np.ndarray | None = None   # float32 [nz][nr]

    @property
    def b_ref(self) -> float:
        """B_z at the origin (used to turn a Hough circle radius into pT)."""
        if self.kind == "uniform":
            return float(self.bz)
        return float(_bilinear_table(self.r0, self.r1, self.z0, self.z1, self.nr, self.nz,
                                     self.br_grid.astype(np.float64), self.bz_grid.astype(np.float64),
                                     np.zeros(1), np.zeros(1))[1][0])


def uniform_field(bz: float = 1.0) -> Field:
    return Field(kind="uniform", bz=float(bz))


def _loop_field(a, zl, r, z):
    """Field of a unit circular current loop (radius a, at height zl); units mu0*I = 1.

    Standard complete-elliptic-integral form; B_r is set to 0 on the axis.
    """
    from scipy.special import ellipe, ellipk
    zeta = z - zl
    al2 = a * a + r * r + zeta * zeta - 2.0 * a * r
    be2 = a * a + r * r + zeta * zeta + 2.0 * a * r
    be = np.sqrt(be2)
    m = 1.0 - al2 / be2
    K = ellipk(m)
    E = ellipe(m)
    c = 1.0 / np.pi
    bz = c / (2.0 * al2 * be) * ((a * a - r * r - zeta * zeta) * E + al2 * K)
    with np.errstate(divide="ignore", invalid="ignore"):
        br = c * zeta / (2.0 * al2 * be * r) * ((a * a + r * r + zeta * zeta) * E - al2 * K)
    br = np.where(r < 1e-9, 0.0, br)
    return br, bz


def solenoid_rz(r: np.ndarray, z: np.ndarray, a: float = 1000.0, ls: float = 1443.0,
                n_nodes: int = 400) -> tuple[np.ndarray, np.ndarray]:
    """Finite current-sheet solenoid (radius a, half-length ls), normalised to B_z(0,0) = 1 T.

    Gauss-Legendre superposition of circular loops. With ls = 1443 mm the on-axis
    field falls by 10 % at |z| = 750 mm.
    """
    r = np.asarray(r, dtype=np.float64).ravel()
    z = np.asarray(z, dtype=np.float64).ravel()
    xg, wg = np.polynomial.legendre.leggauss(n_nodes)
    zl = xg * ls
    w = wg * ls
    br = np.zeros_like(r)
    bz = np.zeros_like(r)
    chunk = max(1, 2_000_000 // n_nodes)
    for s in range(0, r.size, chunk):
        rr = r[s:s + chunk, None]
        zz = z[s:s + chunk, None]
        b1, b2 = _loop_field(a, zl[None, :], rr, zz)
        br[s:s + chunk] = b1 @ w
        bz[s:s + chunk] = b2 @ w
    # the loop sum integrates a^2 / (2 (a^2 + z'^2)^1.5) dz' on the axis; at the origin:
    b00 = ls / math.sqrt(ls * ls + a * a)
    return br / b00, bz / b00


def _grid_nodes(nr, nz, r0, r1, z0, z1):
    rn = r0 + (r1 - r0) * np.arange(nr) / (nr - 1)
    zn = z0 + (z1 - z0) * np.arange(nz) / (nz - 1)
    return rn, zn


def solenoid_field(nr: int = 65, nz: int = 129, r0: float = 0.0, r1: float = 900.0,
                   z0: float = -1000.0, z1: float = 1000.0) -> Field:
    """The finite-solenoid map sampled on a 65x129 (r, z) grid, FP32, B_r(r=0) = 0 exactly."""
    rn, zn = _grid_nodes(nr, nz, r0, r1, z0, z1)
    R, Z = np.meshgrid(rn, zn)       # [nz][nr]
    br, bz = solenoid_rz(R, Z)
    br = br.reshape(nz, nr)
    bz = bz.reshape(nz, nr)
    br[:, 0] = 0.0
    return Field("rz", 0.0, nr, nz, r0, r1, z0, z1, br.astype(np.float32), bz.astype(np.float32))


def linear_bottle_field(b: float, bz0: float = 1.0, nr: int = 65, nz: int = 129, r0: float = 0.0,
                        r1: float = 900.0, z0: float = -1000.0, z1: float = 1000.0) -> Field:
    """B_z = bz0 + b z, B_r = -b r / 2 on the grid (divergence- and curl-free).

    Both components are linear in (r, z), so bilinear interpolation reproduces the
    field exactly inside the grid; its vector potential is A_phi = r (bz0 + b z) / 2.
    Node values are stored as float32; choose b so they are exactly representable
    if exactness of the nodes matters.
    """
    rn, zn = _grid_nodes(nr, nz, r0, r1, z0, z1)
    R, Z = np.meshgrid(rn, zn)
    return Field("rz", 0.0, nr, nz, r0, r1, z0, z1, (-0.5 * b * R).astype(np.float32),
                 (bz0 + b * Z).astype(np.float32))


def constant_grid_field(bz: float = 1.0, nr: int = 65, nz: int = 129) -> Field:
    rn, zn = _grid_nodes(nr, nz, 0.0, 900.0, -1000.0, 1000.0)
    return Field("rz", 0.0, nr, nz, 0.0, 900.0, -1000.0, 1000.0,
                 np.zeros((nz, nr), np.float32), np.full((nz, nr), bz, np.float32))


def _bilinear_table(r0, r1, z0, z1, nr, nz, brg, bzg, r, z):
    """Clamped bilinear lookup into a [nz][nr] table (the simulation's own field model)."""
    dr = (r1 - r0) / (nr - 1)
    dz = (z1 - z0) / (nz - 1)
    u = (r - r0) / dr
    v = (z - z0) / dz
    i = np.clip(np.floor(u), 0, nr - 2).astype(np.int64)
    j = np.clip(np.floor(v), 0, nz - 2).astype(np.int64)
    f = np.clip(u - i, 0.0, 1.0)
    g = np.clip(v - j, 0.0, 1.0)
    def lerp(t):
        return ((1 - g) * ((1 - f) * t[j, i] + f * t[j, i + 1])
                + g * ((1 - f) * t[j + 1, i] + f * t[j + 1, i + 1]))
    return lerp(brg), lerp(bzg)


class TruthField:
    """The simulation's field: exact uniform, or a fine (4x) table of the analytic solenoid."""

    def __init__(self, field: Field, fine: int = 4):
        self.kind = field.kind
        self.bz = field.bz
        if field.kind == "rz":
            self.is_solenoid = _looks_like_solenoid(field)
            if self.is_solenoid:
                nr = (field.nr - 1) * fine + 1
                nz = (field.nz - 1) * fine + 1
                rn, zn = _grid_nodes(nr, nz, field.r0, field.r1, field.z0, field.z1)
                R, Z = np.meshgrid(rn, zn)
                br, bzz = solenoid_rz(R, Z)
                br = br.reshape(nz, nr); bzz = bzz.reshape(nz, nr)
                br[:, 0] = 0.0
                self.tab = (field.r0, field.r1, field.z0, field.z1, nr, nz, br, bzz)
            else:
                self.tab = (field.r0, field.r1, field.z0, field.z1, field.nr, field.nz,
                            field.br_grid.astype(np.float64), field.bz_grid.astype(np.float64))

    def __call__(self, x, y, z):
        if self.kind == "uniform":
            return np.zeros_like(x), np.zeros_like(x), np.full_like(x, self.bz)
        r = np.hypot(x, y)
        br, bz = _bilinear_table(*self.tab, r, z)
        with np.errstate(divide="ignore", invalid="ignore"):
            cx = np.where(r > 1e-9, x / r, 0.0)
            cy = np.where(r > 1e-9, y / r, 0.0)
        return br * cx, br * cy, bz


def _looks_like_solenoid(field: Field) -> bool:
    # The solenoid map is the only non-linear map this module makes; a linear or
    # constant map is simulated with its own (exact) bilinear interpolant.
    bz = field.bz_grid.astype(np.float64)
    return bool(np.ptp(bz[:, field.nr // 2]) > 1e-3 and
                abs(bz[field.nz // 2, 0] - 1.0) < 1e-3 and
                abs(bz[-1, 0] - bz[0, 0]) < 1e-6)


# --------------------------------------------------------------------------------------
# Truth tracks
# --------------------------------------------------------------------------------------
def _helix(x0, t0, a, s):
    """Exact helix in B = B z^, a = kappa q B / |p| (per-sample arc lengths s)."""
    s = np.asarray(s, np.float64)
    sa = np.sin(a * s); ca = np.cos(a * s)
    tx = t0[0] * ca + t0[1] * sa
    ty = t0[1] * ca - t0[0] * sa
    x = x0[0] + (t0[0] * sa + t0[1] * (1.0 - ca)) / a
    y = x0[1] + (t0[1] * sa + t0[0] * (ca - 1.0)) / a
    z = x0[2] + t0[2] * s
    return np.stack([x, y, z], -1), np.stack([tx, ty, np.full_like(s, t0[2])], -1)


def _rk4_tracks(tf, x0, t0, lam, h, n):
    """Classical RK4 of dx/ds = T, dT/ds = lam T x B, vectorised over tracks; returns [n+1, k, 3]."""
    k = x0.shape[0]
    xs = np.empty((n + 1, k, 3)); ts = np.empty((n + 1, k, 3))
    x = x0.copy(); t = t0.copy()
    xs[0] = x; ts[0] = t

    def acc(xx, tt):
        bx, by, bz = tf(xx[:, 0], xx[:, 1], xx[:, 2])
        return lam[:, None] * np.stack([tt[:, 1] * bz - tt[:, 2] * by,
                                        tt[:, 2] * bx - tt[:, 0] * bz,
                                        tt[:, 0] * by - tt[:, 1] * bx], -1)
    for i in range(n):
        a1t = acc(x, t)
        a2x = t + 0.5 * h * a1t; a2t = acc(x + 0.5 * h * t, a2x)
        a3x = t + 0.5 * h * a2t; a3t = acc(x + 0.5 * h * a2x, a3x)
        a4x = t + h * a3t; a4t = acc(x + h * a3x, a4x)
        x = x + h / 6.0 * (t + 2 * a2x + 2 * a3x + a4x)
        t = t + h / 6.0 * (a1t + 2 * a2t + 2 * a3t + a4t)
        xs[i + 1] = x; ts[i + 1] = t
    return xs, ts


def _hermite(x0, t0, x1, t1, h, u):
    """Cubic Hermite position at fraction u in [0,1] of an interval of length h."""
    u = np.asarray(u, np.float64)
    u2 = u * u; u3 = u2 * u
    h00 = 2 * u3 - 3 * u2 + 1; h10 = u3 - 2 * u2 + u; h01 = -2 * u3 + 3 * u2; h11 = u3 - u2
    return (h00[..., None] * x0 + (h10 * h)[..., None] * t0 + h01[..., None] * x1
            + (h11 * h)[..., None] * t1)


@dataclasses.dataclass
class Trajectory:
    """One truth track: samples s (arc length from the seed point), x[n,3], t[n,3].

    pos(s) evaluates the continuous track: the exact helix in a uniform field, the
    cubic Hermite interpolant of the RK4 samples otherwise.
    """
    s: np.ndarray
    x: np.ndarray
    t: np.ndarray
    seed: np.ndarray          # (theta0, z0, px0, py0, pz0) at the first outward crossing of R0
    p: float
    q: float
    helix: tuple | None = None  # (x_seed, t_seed, a) when exact

    def pos(self, s):
        s = np.asarray(s, np.float64)
        if self.helix is not None:
            return _helix(self.helix[0], self.helix[1], self.helix[2], s)[0]
        h = self.s[1] - self.s[0]
        k = np.clip(np.floor((s - self.s[0]) / h).astype(np.int64), 0, self.s.size - 2)
        u = (s - self.s[k]) / h
        return _hermite(self.x[k], self.t[k], self.x[k + 1], self.t[k + 1], h, u)


def trace_truth(tf: TruthField, vertex: np.ndarray, pvec: np.ndarray, q: float, s_after: float,
                h: float = 0.5) -> list[Trajectory | None]:
    """Trace tracks from their vertices; keep samples from the seed point on.

    The seed point is the first outward crossing of r = R0, located by bisection
    (on the exact helix, or on the Hermite interpolant) to ~1e-9 mm. Tracks that
    never reach R0 give None.
    """
    vertex = np.atleast_2d(vertex).astype(np.float64)
    pvec = np.atleast_2d(pvec).astype(np.float64)
    k = vertex.shape[0]
    pm = np.linalg.norm(pvec, axis=1)
    t0 = pvec / pm[:, None]
    lam = KAPPA * q / pm
    s_before = 1200.0                       # enough path to reach R0 from |r| < 100 mm
    n = int(math.ceil((s_before + s_after) / h)) + 2
    s_all = np.arange(n + 1) * h
    if tf.kind == "uniform":
        xs = np.empty((n + 1, k, 3)); ts = np.empty((n + 1, k, 3))
        for i in range(k):
            xs[:, i], ts[:, i] = _helix(vertex[i], t0[i], lam[i] * tf.bz, s_all)
    else:
        xs, ts = _rk4_tracks(tf, vertex, t0, lam, h, n)
    out: list[Trajectory | None] = []
    for i in range(k):
        x = xs[:, i]; t = ts[:, i]
        r2 = x[:, 0] ** 2 + x[:, 1] ** 2
        idx = np.nonzero((r2[:-1] < R0_SEED ** 2) & (r2[1:] >= R0_SEED ** 2))[0]
        if idx.size == 0 or idx[0] * h > s_before:
            out.append(None); continue
        j = int(idx[0])
        exact = tf.kind == "uniform"
        a_i = lam[i] * tf.bz if exact else 0.0

        def at(sv):
            if exact:
                return _helix(vertex[i], t0[i], a_i, np.array([sv]))
            u = np.array((sv - j * h) / h)
            return _hermite(x[j], t[j], x[j + 1], t[j + 1], h, u)[None, :], None
        lo, hi = j * h, (j + 1) * h
        for _ in range(70):
            mid = 0.5 * (lo + hi)
            pm_ = at(mid)[0][0]
            if pm_[0] ** 2 + pm_[1] ** 2 < R0_SEED ** 2:
                lo = mid
            else:
                hi = mid
        s_seed = 0.5 * (lo + hi)
        if exact:
            xsd, tsd = _helix(vertex[i], t0[i], a_i, np.array([s_seed]))
            xseed, tseed = xsd[0], tsd[0]
        else:
            uu = (s_seed - j * h) / h
            xseed = _hermite(x[j], t[j], x[j + 1], t[j + 1], h, np.array(uu))
            d00 = 6 * uu * uu - 6 * uu; d10 = 3 * uu * uu - 4 * uu + 1; d01 = -d00; d11 = 3 * uu * uu - 2 * uu
            tseed = (d00 * x[j] + d10 * h * t[j] + d01 * x[j + 1] + d11 * h * t[j + 1]) / h
            tseed = tseed / np.linalg.norm(tseed)
        keep = slice(j, None)
        theta0 = math.atan2(xseed[1], xseed[0])
        pseed = pm[i] * tseed
        seed = np.array([theta0, xseed[2], pseed[0], pseed[1], pseed[2]])
        out.append(Trajectory(s_all[keep] - s_seed, x[keep].copy(), t[keep].copy(), seed,
                              float(pm[i]), q, (xseed, tseed, a_i) if exact else None))
    return out


# --------------------------------------------------------------------------------------
# Hits: true distance of each wire to the continuous trajectory
# --------------------------------------------------------------------------------------
def _point_segment_dist(p, m, u, L):
    r = p - m
    t = np.clip(np.einsum("...k,...k->...", r, u), -L, L)
    v = r - t[..., None] * u
    return np.sqrt(np.einsum("...k,...k->...", v, v))


def true_wire_distances(geo: Geometry, tr: Trajectory, s_max: float, reach: float = 8.0):
    """All wires within `reach` mm of the track for s in [0, s_max].

    Returns (wire ids, true distance, arc length of the closest approach), one entry per
    wire (the global minimum over all passes), ordered by arc length.
    """
    h = tr.s[1] - tr.s[0]
    keep = (tr.s >= -h) & (tr.s <= s_max + h)
    x = tr.x[keep]; s = tr.s[keep]
    r = np.hypot(x[:, 0], x[:, 1])
    G, D, S = [], [], []
    for l in range(geo.n_layers):
        band = (r > geo.layer_rmin[l] - reach - 2.0) & (r < geo.layer_rmax[l] + reach + 2.0)
        band &= np.abs(x[:, 2]) < geo.half_z + reach + 2.0
        idx = np.nonzero(band)[0]
        if idx.size == 0:
            continue
        n = int(geo.layer_nwires[l]); rl = geo.layer_radius[l]; a = geo.layer_stereo[l]
        p = x[idx]
        phi_p = np.arctan2(p[:, 1], p[:, 0])
        shift = np.arctan2(p[:, 2] * math.tan(a), rl)
        jc = np.round((phi_p - shift) * n / (2 * np.pi) - 0.5 * (l % 2)).astype(np.int64)
        for dj in range(-3, 4):
            g = geo.layer_first[l] + np.mod(jc + dj, n)
            m = np.stack([geo.mx[g], geo.my[g], geo.mz[g]], -1)
            u = np.stack([geo.ux[g], geo.uy[g], geo.uz[g]], -1)
            d = _point_segment_dist(p, m, u, geo.half_len[g])
            ok = d < reach + 1.0
            G.append(g[ok]); D.append(d[ok]); S.append(s[idx][ok])
    if not G:
        z = np.zeros(0)
        return z.astype(np.int32), z, z
    G = np.concatenate(G); D = np.concatenate(D); S = np.concatenate(S)
    if G.size == 0:
        z = np.zeros(0)
        return z.astype(np.int32), z, z
    order = np.lexsort((D, G))
    G, D, S = G[order], D[order], S[order]
    first = np.ones(G.size, bool); first[1:] = G[1:] != G[:-1]
    G, D, S = G[first], D[first], S[first]
    # golden-section refinement of each wire's minimum on the continuous track
    m = np.stack([geo.mx[G], geo.my[G], geo.mz[G]], -1)
    u = np.stack([geo.ux[G], geo.uy[G], geo.uz[G]], -1)
    L = geo.half_len[G]

    def f(sv):
        return _point_segment_dist(tr.pos(sv), m, u, L)
    a_ = S - h; b_ = S + h
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    c_ = b_ - gr * (b_ - a_); d_ = a_ + gr * (b_ - a_)
    fc, fd = f(c_), f(d_)
    for _ in range(48):
        left = fc < fd
        b_ = np.where(left, d_, b_); a_ = np.where(left, a_, c_)
        nc = np.where(left, b_ - gr * (b_ - a_), d_)
        nd = np.where(left, c_, a_ + gr * (b_ - a_))
        nfc_new = f(np.where(left, nc, nd))
        fc, fd = np.where(left, nfc_new, fd), np.where(left, fc, nfc_new)
        c_, d_ = nc, nd
    sv = 0.5 * (a_ + b_)
    dv = np.minimum(f(sv), D)
    ok = (dv <= reach) & (sv >= 0.0) & (sv <= s_max)
    G, dv, sv = G[ok], dv[ok], sv[ok]
    order = np.argsort(sv)
    return G[order].astype(np.int32), dv[order], sv[order]


# --------------------------------------------------------------------------------------
# Events
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Event:
    wire_id: np.ndarray           # int32 [H]
    drift: np.ndarray             # float32 [H], mm
    is_noise: np.ndarray          # bool [H]
    track_of: np.ndarray          # int32 [H], -1 for noise
    true_dist: np.ndarray         # float64 [H], true DOCA (nan for noise)
    truth_seeds: np.ndarray       # [n_tracks, 5]
    truth_p: np.ndarray           # [n_tracks]
    turn_of: np.ndarray | None = None  # int32 [H]: chamber pass of the hit (0 = first), -1 noise


def turn_index(tr: "Trajectory", s_hit: np.ndarray) -> np.ndarray:
    """Truth turn partition of points at arc lengths s_hit: the number of outward
    crossings of r = R0 after the seed crossing that precede them (0 = first pass)."""
    r2 = tr.x[:, 0] ** 2 + tr.x[:, 1] ** 2
    up = (r2[:-1] < R0_SEED ** 2) & (r2[1:] >= R0_SEED ** 2)
    s_cross = tr.s[1:][up]
    s_cross = s_cross[s_cross > 1.0]
    return np.searchsorted(s_cross, np.asarray(s_hit, np.float64), side="right").astype(np.int32)


def _draw_vertex(rng, k):
    rv = 100.0 * np.sqrt(rng.random(k))
    ph = 2 * np.pi * rng.random(k)
    return np.stack([rv * np.cos(ph), rv * np.sin(ph), rng.uniform(-200.0, 200.0, k)], -1)


def _isotropic(rng, k, p):
    c = rng.uniform(-1.0, 1.0, k)
    ph = 2 * np.pi * rng.random(k)
    s = np.sqrt(1 - c * c)
    return np.stack([s * np.cos(ph), s * np.sin(ph), c], -1) * np.asarray(p)[..., None]


def _finish_event(rng, geo, wires, dists, track_of, truths, ps, n_noise, sigma, dmax=8.0, turn_of=None):
    hit_set = set(int(w) for w in wires)
    free = np.array([w for w in range(geo.n_wires) if w not in hit_set], dtype=np.int32)
    noise = rng.choice(free, size=n_noise, replace=False) if n_noise > 0 else np.zeros(0, np.int32)
    drift_true = np.clip(np.asarray(dists) + (rng.normal(0.0, sigma, len(dists)) if sigma > 0 else 0.0),
                         0.0, dmax)
    drift_noise = rng.uniform(0.0, dmax, n_noise)
    wid = np.concatenate([np.asarray(wires, np.int32), noise.astype(np.int32)])
    drift = np.concatenate([drift_true, drift_noise]).astype(np.float32)
    isn = np.concatenate([np.zeros(len(wires), bool), np.ones(n_noise, bool)])
    tro = np.concatenate([np.asarray(track_of, np.int32), np.full(n_noise, -1, np.int32)])
    tdist = np.concatenate([np.asarray(dists, np.float64), np.full(n_noise, np.nan)])
    order = np.argsort(wid, kind="stable")      # hits arrive ordered by wire id
    turns = None
    if turn_of is not None:
        turns = np.concatenate([np.asarray(turn_of, np.int32), np.full(n_noise, -1, np.int32)])[order]
    return Event(wid[order], drift[order], isn[order], tro[order], tdist[order],
                 np.asarray(truths, np.float64).reshape(-1, 5), np.asarray(ps, np.float64), turns)


def event_single_turn(geo: Geometry, field: Field, seed: int, n_hits: int = 40,
                      sigma: float = 0.2, n_steps: int = 2000, p: float = P_SIGNAL) -> Event:
    """One signal e- under one turn in the chamber; the first n_hits hits by arc length."""
    rng = np.random.default_rng([BASE_SEED, 1, seed])
    tf = TruthField(field)
    turn = 2 * np.pi * p / (KAPPA * field.b_ref)
    while True:
        v = _draw_vertex(rng, 8)
        pv = _isotropic(rng, 8, p)
        for tr in trace_truth(tf, v, pv, ELECTRON_Q, min(turn, n_steps - 20.0)):
            if tr is None:
                continue
            w, d, s = true_wire_distances(geo, tr, min(turn, n_steps - 20.0))
            if w.size >= n_hits:
                w, d, s = w[:n_hits], d[:n_hits], s[:n_hits]
                return _finish_event(rng, geo, w, d, np.zeros(n_hits), [tr.seed], [p], 0, sigma,
                                     turn_of=turn_index(tr, s))


def event_multi_turn(geo: Geometry, field: Field, seed: int, n_steps: int = 6000,
                     noise_frac: float = 0.30, sigma: float = 0.2, p: float = P_SIGNAL,
                     true_range=(100, 140), min_passes: int = 2) -> Event:
    """One 2-3 turn signal e- (|pz| ~ U[5,20] MeV/c) with ~120 true hits plus noise."""
    rng = np.random.default_rng([BASE_SEED, 2, seed])
    tf = TruthField(field)
    while True:
        k = 8
        pz = rng.uniform(5.0, 20.0, k) * rng.choice([-1.0, 1.0], k)
        pt = np.sqrt(p * p - pz * pz)
        ph = 2 * np.pi * rng.random(k)
        pv = np.stack([pt * np.cos(ph), pt * np.sin(ph), pz], -1)
        v = _draw_vertex(rng, k)
        for tr in trace_truth(tf, v, pv, ELECTRON_Q, n_steps - 20.0):
            if tr is None:
                continue
            w, d, s = true_wire_distances(geo, tr, n_steps - 20.0)
            # count chamber passes: outward crossings of the first layer radius
            r = np.hypot(tr.x[:, 0], tr.x[:, 1])
            passes = int(np.sum((r[:-1] < geo.layer_rmin[0]) & (r[1:] >= geo.layer_rmin[0])))
            if true_range[0] <= w.size <= true_range[1] and passes >= min_passes:
                n_noise = int(round(noise_frac * w.size))
                return _finish_event(rng, geo, w, d, np.zeros(w.size), [tr.seed], [p], n_noise, sigma,
                                     turn_of=turn_index(tr, s))


def event_fixed_total(geo: Geometry, field: Field, seed: int, n_total: int = 150,
                      noise_frac: float = 0.20, n_steps: int = 6000, sigma: float = 0.2,
                      p: float = P_SIGNAL) -> Event:
    """One signal e- with n_total hits of which round(noise_frac*n_total) are noise."""
    rng = np.random.default_rng([BASE_SEED, 3, seed])
    tf = TruthField(field)
    n_noise = int(round(noise_frac * n_total))
    n_true = n_total - n_noise
    while True:
        k = 8
        pz = rng.uniform(5.0, 20.0, k) * rng.choice([-1.0, 1.0], k)
        pt = np.sqrt(p * p - pz * pz)
        ph = 2 * np.pi * rng.random(k)
        pv = np.stack([pt * np.cos(ph), pt * np.sin(ph), pz], -1)
        v = _draw_vertex(rng, k)
        for tr in trace_truth(tf, v, pv, ELECTRON_Q, n_steps - 20.0):
            if tr is None:
                continue
            w, d, s = true_wire_distances(geo, tr, n_steps - 20.0)
            if w.size >= n_true:
                return _finish_event(rng, geo, w[:n_true], d[:n_true], np.zeros(n_true),
                                     [tr.seed], [p], n_noise, sigma, turn_of=turn_index(tr, s[:n_true]))


def events_batch(geo: Geometry, field: Field, n_events: int = 512, seed: int = 0,
                 n_steps: int = 6000, sigma: float = 0.2, hits_range=(40, 300),
                 noise_range=(0.1, 0.4), p_range=(60.0, 105.0), max_tracks: int = 3,
                 truth_step: float = 1.0) -> list[Event]:
    """Many events: 1-3 e- with p ~ U[60,105] MeV/c, 40-300 hits, 10-40 % noise.

    Each event draws its track count and hit budget from its own generator; the
    tracks are then traced together (vectorised) until every event has its own:
    no track appears in two events.
    """
    rng = np.random.default_rng([BASE_SEED, 4, seed])
    tf = TruthField(field)
    plans = []
    for e in range(n_events):
        er = np.random.default_rng([BASE_SEED, 4, seed, e])
        nt = int(er.integers(1, max_tracks + 1))
        n_total = int(er.integers(hits_range[0], hits_range[1] + 1))
        plans.append((er, nt, n_total, er.uniform(*noise_range)))
    need = sum(nt for _, nt, _, _ in plans)
    pool = []
    while len(pool) < need:
        k = 2 * (need - len(pool)) + 8
        pm = rng.uniform(*p_range, k)
        pz = rng.uniform(-25.0, 25.0, k)
        pz = np.clip(pz, -0.5 * pm, 0.5 * pm)
        pt = np.sqrt(pm * pm - pz * pz)
        ph = 2 * np.pi * rng.random(k)
        pv = np.stack([pt * np.cos(ph), pt * np.sin(ph), pz], -1)
        v = _draw_vertex(rng, k)
        for tr, pmi in zip(trace_truth(tf, v, pv, ELECTRON_Q, n_steps - 20.0, h=truth_step), pm):
            if tr is None or len(pool) >= need:
                continue
            w, d, s = true_wire_distances(geo, tr, n_steps - 20.0)
            if w.size >= 40:
                pool.append((tr.seed, float(pmi), w, d))
    events = []
    first = 0
    for er, nt, n_total, f in plans:
        picks = range(first, first + nt)
        first += nt
        n_noise = int(round(f * n_total))
        n_true = n_total - n_noise
        # round-robin by arc length across tracks, one hit per wire (smallest distance)
        per = [list(zip(pool[i][2].tolist(), pool[i][3].tolist())) for i in picks]
        chosen: dict[int, tuple[float, int]] = {}
        pos = [0] * nt
        while len(chosen) < n_true and any(pos[t] < len(per[t]) for t in range(nt)):
            for t in range(nt):
                if pos[t] < len(per[t]) and len(chosen) < n_true:
                    wv, dv = per[t][pos[t]]; pos[t] += 1
                    if wv not in chosen or dv < chosen[wv][0]:
                        chosen[wv] = (dv, t)
        wires = np.array(list(chosen.keys()), dtype=np.int32)
        dists = np.array([chosen[w][0] for w in wires])
        tro = np.array([chosen[w][1] for w in wires], dtype=np.int32)
        # keep the drawn noise fraction when the tracks give fewer true hits than asked
        n_noise = n_noise if wires.size == n_true else int(round(f / (1.0 - f) * wires.size))
        events.append(_finish_event(er, geo, wires, dists, tro, [pool[i][0] for i in picks],
                                    [pool[i][1] for i in picks], n_noise, sigma))
    return events


def events_multi_turn(geo: Geometry, field: Field, n_events: int, seed: int = 0, n_steps: int = 6000,
                      noise_frac: float = 0.30, sigma: float = 0.2, p: float = P_SIGNAL,
                      true_range=(100, 140), min_passes: int = 2, truth_step: float = 1.0) -> list[Event]:
    """Many multi-turn events as event_multi_turn makes one (one 2-3 pass e- with
    |pz| ~ U[5,20] MeV/c, 100-140 true hits, 30 % noise, per-hit true pass), with the
    candidate tracks traced together."""
    rng = np.random.default_rng([BASE_SEED, 5, seed])
    tf = TruthField(field)
    events: list[Event] = []
    while len(events) < n_events:
        k = 8 * (n_events - len(events)) + 8
        pz = rng.uniform(5.0, 20.0, k) * rng.choice([-1.0, 1.0], k)
        pt = np.sqrt(p * p - pz * pz)
        ph = 2 * np.pi * rng.random(k)
        pv = np.stack([pt * np.cos(ph), pt * np.sin(ph), pz], -1)
        v = _draw_vertex(rng, k)
        for tr in trace_truth(tf, v, pv, ELECTRON_Q, n_steps - 20.0, h=truth_step):
            if tr is None or len(events) >= n_events:
                continue
            r = np.hypot(tr.x[:, 0], tr.x[:, 1])
            passes = int(np.sum((r[:-1] < geo.layer_rmin[0]) & (r[1:] >= geo.layer_rmin[0])))
            if passes < min_passes:
                continue
            w, d, s = true_wire_distances(geo, tr, n_steps - 20.0)
            if true_range[0] <= w.size <= true_range[1]:
                n_noise = int(round(noise_frac * w.size))
                events.append(_finish_event(rng, geo, w, d, np.zeros(w.size), [tr.seed], [p], n_noise, sigma,
                                            turn_of=turn_index(tr, s)))
    return events


def pack_events(events: list[Event]):
    """CSR layout for the hit upload: (ev_off[E+1] int32, wire_id[H] int32, drift[H] float32)."""
    off = np.zeros(len(events) + 1, dtype=np.int32)
    off[1:] = np.cumsum([e.wire_id.size for e in events])
    wid = np.concatenate([e.wire_id for e in events]).astype(np.int32) if events else np.zeros(0, np.int32)
    dr = np.concatenate([e.drift for e in events]).astype(np.float32) if events else np.zeros(0, np.float32)
    return off, wid, dr


# --------------------------------------------------------------------------------------
# Seed windows (inputs of the scan when no Hough stage is used)
# --------------------------------------------------------------------------------------
WINDOW_DTYPE = np.dtype([("event", "<i4"), ("candidate", "<i4"), ("center", "<f8", (5,)),
                         ("half_width", "<f8", (5,)), ("count", "<i4", (5,)), ("pad", "<i4")])


def make_windows(rows) -> np.ndarray:
    """rows: iterable of (event, candidate, center5, half_width5, count5)."""
    rows = list(rows)
    w = np.zeros(len(rows), dtype=WINDOW_DTYPE)
    for i, (ev, cand, c, hw, n) in enumerate(rows):
        w[i]["event"] = ev; w[i]["candidate"] = cand
        w[i]["center"] = c; w[i]["half_width"] = hw; w[i]["count"] = n
    return w


def random_seeds(rng: np.random.Generator, center, half_width, n: int) -> np.ndarray:
    """n seeds drawn uniformly in a 5-D box (used for explicit-seed scans and tests)."""
    c = np.asarray(center, np.float64); w = np.asarray(half_width, np.float64)
    return c + w * rng.uniform(-1.0, 1.0, (n, 5))
