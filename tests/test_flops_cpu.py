"""The flop model of the roofline (flops.py) against an operation count of the step
and distance formulas re-expressed here (add/sub/mul/div/sqrt = 1, an FMA = its mul
and add): the fourth-order Nystrom step (section 2.2) in a uniform field and in the
(r, z) map with its three bilinear field evaluations, and the exact chord/wire
distance. Counting choices (negations, per-launch constants, clamps) move a count by
a few flops, so each is checked to within 3."""
import math


class N:
    """A number that counts the arithmetic operations applied to it."""
    n = 0

    def __init__(self, v):
        self.v = v

    @staticmethod
    def _w(o):
        return o if isinstance(o, N) else N(o)

    def __add__(self, o):
        N.n += 1
        return N(self.v + self._w(o).v)

    __radd__ = __add__

    def __sub__(self, o):
        N.n += 1
        return N(self.v - self._w(o).v)

    def __rsub__(self, o):
        N.n += 1
        return N(self._w(o).v - self.v)

    def __mul__(self, o):
        N.n += 1
        return N(self.v * self._w(o).v)

    __rmul__ = __mul__

    def __truediv__(self, o):
        N.n += 1
        return N(self.v / self._w(o).v)

    def __neg__(self):
        return N(-self.v)


def rkn_uniform(x, y, z, tx, ty, tz, lam, bz, h):
    h2 = 0.5 * h; hh6 = h * h / 6; h6 = h / 6       # constants per launch, not per step
    a = lam * bz
    k1x = a * ty; k1y = -(a * tx)
    t2x = tx + h2 * k1x; t2y = ty + h2 * k1y
    k2x = a * t2y; k2y = -(a * t2x)
    t3x = tx + h2 * k2x; t3y = ty + h2 * k2y
    k3x = a * t3y; k3y = -(a * t3x)
    t4x = tx + h * k3x; t4y = ty + h * k3y
    k4x = a * t4y; k4y = -(a * t4x)
    dx = h * tx + hh6 * (k1x + k2x + k3x)
    dy = h * ty + hh6 * (k1y + k2y + k3y)
    dz = h * tz
    tx = tx + h6 * (k1x + 2 * (k2x + k3x) + k4x)
    ty = ty + h6 * (k1y + 2 * (k2y + k3y) + k4y)
    return x + dx, y + dy, z + dz, tx, ty

def field(x, y, z):
    r2 = x * x + y * y
    inv_r = N(1.0 / math.sqrt(r2.v)); N.n += 1       # one rsqrt
    r = r2 * inv_r
    u = r * 0.1 + (-1.0); v = z * 0.1 + (-1.0)       # fma each
    a = u - 3.0; b = v - 4.0                          # cell fractions
    n00x, n01x, n10x, n11x = N(1.), N(1.), N(1.), N(1.)
    n00y, n01y, n10y, n11y = N(1.), N(1.), N(1.), N(1.)
    br0 = a * (n01x - n00x) + n00x; br1 = a * (n11x - n10x) + n10x
    bz0 = a * (n01y - n00y) + n00y; bz1 = a * (n11y - n10y) + n10y
    br = b * (br1 - br0) + br0; bz = b * (bz1 - bz0) + bz0
    s = br * inv_r
    return s * x, s * y, bz

def rkn_grid(x, y, z, tx, ty, tz, l, h):
    h2 = 0.5 * h; hh6 = h * h / 6; h6 = h / 6; hh8 = h * h * 0.125; hh2 = h * h * 0.5
    bx, by, bz = field(x, y, z)
    k1x = l * (ty * bz - tz * by); k1y = l * (tz * bx - tx * bz); k1z = l * (tx * by - ty * bx)
    bx, by, bz = field(x + h2 * tx + hh8 * k1x, y + h2 * ty + hh8 * k1y, z + h2 * tz + hh8 * k1z)
    t2x = tx + h2 * k1x; t2y = ty + h2 * k1y; t2z = tz + h2 * k1z
    lbx = l * bx; lby = l * by; lbz = l * bz
    k2x = t2y * lbz - t2z * lby; k2y = t2z * lbx - t2x * lbz; k2z = t2x * lby - t2y * lbx
    t3x = tx + h2 * k2x; t3y = ty + h2 * k2y; t3z = tz + h2 * k2z
    k3x = t3y * lbz - t3z * lby; k3y = t3z * lbx - t3x * lbz; k3z = t3x * lby - t3y * lbx
    bx, by, bz = field(x + h * tx + hh2 * k3x, y + h * ty + hh2 * k3y, z + h * tz + hh2 * k3z)
    t4x = tx + h * k3x; t4y = ty + h * k3y; t4z = tz + h * k3z
    k4x = l * (t4y * bz - t4z * by); k4y = l * (t4z * bx - t4x * bz); k4z = l * (t4x * by - t4y * bx)
    dx = h * tx + hh6 * (k1x + k2x + k3x); dy = h * ty + hh6 * (k1y + k2y + k3y); dz = h * tz + hh6 * (k1z + k2z + k3z)
    tx = tx + h6 * (k1x + 2 * (k2x + k3x) + k4x); ty = ty + h6 * (k1y + 2 * (k2y + k3y) + k4y)
    tz = tz + h6 * (k1z + 2 * (k2z + k3z) + k4z)
    return x + dx, y + dy, z + dz

def seg_wire(p0, p1, m, u, L):
    dx, dy, dz = p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]
    rx, ry, rz = p0[0] - m[0], p0[1] - m[1], p0[2] - m[2]
    a = dx * dx + dy * dy + dz * dz
    b = dx * u[0] + dy * u[1] + dz * u[2]
    e = dx * rx + dy * ry + dz * rz
    f = u[0] * rx + u[1] * ry + u[2] * rz
    den = a - b * b
    s = (b * f - e) * (N(1.0) / den)      # rcp + mul
    t = b * s + f
    vx = rx + s * dx - t * u[0]; vy = ry + s * dy - t * u[1]; vz = rz + s * dz - t * u[2]
    return vx * vx + vy * vy + vz * vz



def _v(*a):
    return [N(x) for x in a]


def test_flop_model_matches_counted_formulas():
    from paper_1908_01949_amd import flops
    N.n = 0
    rkn_uniform(*_v(500, 0, 0, 0.6, 0.8, 0.0, -0.003, 1.0), 1.0)
    assert abs(N.n - flops.F_RKN_UNIFORM) <= 3, N.n
    N.n = 0
    field(*_v(500.0, 10.0, 5.0))
    assert abs(N.n - flops.F_FIELD) <= 3, N.n
    N.n = 0
    rkn_grid(*_v(500, 10, 5, 0.6, 0.8, 0.0, -0.003), 1.0)
    assert abs(N.n - flops.F_RKN_GRID) <= 3, N.n
    N.n = 0
    seg_wire(_v(500, 0, 0), _v(501, 0.5, 0.1), _v(530, 1, 0), _v(0, 0.07, 0.99), 750.0)
    assert abs(N.n - flops.F_DOCA) <= 3, N.n
