"""Seeded synthetic inputs for the HPS workloads.

This module draws random parameters and evaluates coefficient, source and
boundary-data *functions of position* at points that the caller supplies.  It
holds none of the solver's arithmetic (no differentiation, interpolation,
factorization or merge): both the CPU oracle and the GPU library consume the
arrays it returns, and it imports neither of them.

Seeding: workload ``c`` uses ``numpy.random.default_rng([1000 + c, k])`` for its
k-th independent stream, so every array is reproducible from (config, stream).

Coefficient layout (shared by every consumer): ``coeffs[leaf, term, point]``
with point order of the caller's point array.  Term order (the operator is
``L u = sum_t c_t(x) d_t u``):

* 2D: ``c_xx, c_xy, c_yy, c_x, c_y, c_0``  (6 terms)
* 3D: ``c_xx, c_yy, c_zz, c_xy, c_xz, c_yz, c_x, c_y, c_z, c_0``  (10 terms)
"""
from __future__ import annotations

import numpy as np

TERMS_2D = ("xx", "xy", "yy", "x", "y", "0")
TERMS_3D = ("xx", "yy", "zz", "xy", "xz", "yz", "x", "y", "z", "0")


def n_terms(dim: int) -> int:
    return 6 if dim == 2 else 10


def rng(config: int, stream: int = 0) -> np.random.Generator:
    """Independent seeded stream ``stream`` of workload ``config``."""
    return np.random.default_rng([1000 + int(config), int(stream)])


def _empty_coeffs(pts: np.ndarray) -> np.ndarray:
    nl, npts, dim = pts.shape
    return np.zeros((nl, n_terms(dim), npts), dtype=np.float64)


def _term(dim: int, name: str) -> int:
    return (TERMS_2D if dim == 2 else TERMS_3D).index(name)


# --------------------------------------------------------------------------
# Gaussian-bump fields (scattering potential q, sources)
# --------------------------------------------------------------------------
def draw_bumps(g: np.random.Generator, nbumps: int = 8, amp=(0.0, 0.5),
               box: float = 0.75, dim: int = 2):
    """Centres ~ U([-box, box]^dim), amplitudes ~ U(amp)."""
    centres = g.uniform(-box, box, size=(nbumps, dim))
    amps = g.uniform(amp[0], amp[1], size=nbumps)
    return {"centres": centres, "amps": amps}


def eval_bumps(params, pts: np.ndarray, width: float = 0.1) -> np.ndarray:
    """sum_b A_b exp(-|x - z_b|^2 / (2 width^2)) at ``pts[..., dim]``."""
    x = np.asarray(pts, dtype=np.float64)
    out = np.zeros(x.shape[:-1])
    for z, a in zip(params["centres"], params["amps"]):
        r2 = np.sum((x - z) ** 2, axis=-1)
        out += a * np.exp(-r2 / (2.0 * width * width))
    return out


def draw_source_bump(g: np.random.Generator, box: float = 0.75, dim: int = 2):
    """One source bump: centre ~ U([-box, box]^dim), amplitude ~ N(0, 1)."""
    return {"centres": g.uniform(-box, box, size=(1, dim)),
            "amps": g.normal(0.0, 1.0, size=1)}


# --------------------------------------------------------------------------
# Boundary data: Fourier series in perimeter arclength of [-1, 1]^2
# --------------------------------------------------------------------------
def draw_fourier(g: np.random.Generator, modes: int = 16):
    m = np.arange(modes + 1)
    sd = 1.0 / (1.0 + m)
    return {"a": g.normal(0.0, 1.0, size=modes + 1) * sd,
            "b": g.normal(0.0, 1.0, size=modes + 1) * sd}


def perimeter_arclength(pts: np.ndarray) -> np.ndarray:
    """Counter-clockwise arclength s in [0, 8) of points on the boundary of
    [-1, 1]^2, starting at (-1, -1): bottom, right, top, left."""
    x, y = pts[..., 0], pts[..., 1]
    s = np.empty(x.shape)
    tol = 1e-12
    bot = np.abs(y + 1) < tol
    rig = (~bot) & (np.abs(x - 1) < tol)
    top = (~bot) & (~rig) & (np.abs(y - 1) < tol)
    lef = ~(bot | rig | top)
    s[bot] = x[bot] + 1.0
    s[rig] = 2.0 + (y[rig] + 1.0)
    s[top] = 4.0 + (1.0 - x[top])
    s[lef] = 6.0 + (1.0 - y[lef])
    return s


def eval_fourier(params, pts: np.ndarray) -> np.ndarray:
    s = perimeter_arclength(pts)
    out = np.zeros(s.shape)
    for m, (am, bm) in enumerate(zip(params["a"], params["b"])):
        w = 2.0 * np.pi * m * s / 8.0
        out += am * np.cos(w) + bm * np.sin(w)
    return out


# --------------------------------------------------------------------------
# Operators
# --------------------------------------------------------------------------
def coeffs_poisson(pts: np.ndarray) -> np.ndarray:
    """-Laplace u: c_xx = c_yy (= c_zz) = -1."""
    c = _empty_coeffs(pts)
    dim = pts.shape[-1]
    for name in ("xx", "yy", "zz")[:dim]:
        c[:, _term(dim, name), :] = -1.0
    return c


def coeffs_helmholtz(pts: np.ndarray, k: float, q: np.ndarray) -> np.ndarray:
    """-Laplace u - k^2 (1 + q(x)) u, with q sampled at ``pts`` (shape
    [leaf, point])."""
    c = coeffs_poisson(pts)
    c[:, _term(pts.shape[-1], "0"), :] = -(k * k) * (1.0 + q)
    return c


def coeffs_general2d(pts: np.ndarray, fields: dict) -> np.ndarray:
    """Arbitrary 2D coefficients given as callables of (x, y)."""
    c = _empty_coeffs(pts)
    x, y = pts[..., 0], pts[..., 1]
    for name, fn in fields.items():
        c[:, _term(2, name), :] = fn(x, y)
    return c


# 3D variable-coefficient Poisson  div(a grad u) = f, expanded as
# a * Laplace u + grad a . grad u  (a = 1 + 0.5 prod_i sin(k_i pi x_i + phi_i)).
def draw_sinprod(g: np.random.Generator, dim: int = 3):
    return {"k": g.integers(1, 4, size=dim).astype(np.float64),
            "phi": g.uniform(0.0, 2.0 * np.pi, size=dim)}


def eval_sinprod(params, pts: np.ndarray):
    """Returns a(x) and grad a(x) (shape [..., dim])."""
    x = np.asarray(pts)
    k, phi = params["k"], params["phi"]
    arg = k * np.pi * x + phi
    s, c = np.sin(arg), np.cos(arg)
    prod = np.prod(s, axis=-1)
    a = 1.0 + 0.5 * prod
    grad = np.empty(x.shape)
    dim = x.shape[-1]
    for i in range(dim):
        others = np.prod(np.delete(s, i, axis=-1), axis=-1)
        grad[..., i] = 0.5 * k[i] * np.pi * c[..., i] * others
    return a, grad


def coeffs_divgrad(pts: np.ndarray, params) -> np.ndarray:
    dim = pts.shape[-1]
    a, grad = eval_sinprod(params, pts)
    c = _empty_coeffs(pts)
    for name in ("xx", "yy", "zz")[:dim]:
        c[:, _term(dim, name), :] = a
    for i, name in enumerate(("x", "y", "z")[:dim]):
        c[:, _term(dim, name), :] = grad[..., i]
    return c


# --------------------------------------------------------------------------
# Manufactured solutions (closed forms) used as test data
# --------------------------------------------------------------------------
def sinsin(pts):
    x, y = pts[..., 0], pts[..., 1]
    return np.sin(np.pi * x) * np.sin(np.pi * y)


def sinsin_minus_laplacian(pts):
    """-Laplace of sin(pi x) sin(pi y)."""
    return 2.0 * np.pi ** 2 * sinsin(pts)


def sin3_plus_xyz(pts):
    """u = sin(pi x) sin(pi y) sin(pi z) + x y z and its gradient/Laplacian."""
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    u = sx * sy * sz + x * y * z
    grad = np.stack([np.pi * cx * sy * sz + y * z,
                     np.pi * sx * cy * sz + x * z,
                     np.pi * sx * sy * cz + x * y], axis=-1)
    lap = -3.0 * np.pi ** 2 * sx * sy * sz
    return u, grad, lap


def divgrad_source(params, pts):
    """f = div(a grad u) = a Laplace u + grad a . grad u for u = sin3_plus_xyz."""
    a, ga = eval_sinprod(params, pts)
    _, gu, lap = sin3_plus_xyz(pts)
    return a * lap + np.sum(ga * gu, axis=-1)


def dtn_problem_u(pts):
    """Manufactured solution of the variable-coefficient Poisson test problem
    (Section 5.1): u = e^{5x} sin(5y) + sin(10 pi x) sin(pi y)."""
    x, y = pts[..., 0], pts[..., 1]
    return np.exp(5 * x) * np.sin(5 * y) + np.sin(10 * np.pi * x) * np.sin(np.pi * y)


def dtn_problem_coeffs(pts):
    """Laplace u - cos(5y) u_x + sin(5y) u_y (Section 5.1)."""
    return coeffs_general2d(pts, {
        "xx": lambda x, y: np.ones_like(x),
        "yy": lambda x, y: np.ones_like(x),
        "x": lambda x, y: -np.cos(5 * y),
        "y": lambda x, y: np.sin(5 * y),
    })


def dtn_problem_f(pts):
    x, y = pts[..., 0], pts[..., 1]
    e = np.exp(5 * x)
    s10, c10 = np.sin(10 * np.pi * x), np.cos(10 * np.pi * x)
    sy, cy = np.sin(np.pi * y), np.cos(np.pi * y)
    u_xx = 25 * e * np.sin(5 * y) - (10 * np.pi) ** 2 * s10 * sy
    u_yy = -25 * e * np.sin(5 * y) - np.pi ** 2 * s10 * sy
    u_x = 5 * e * np.sin(5 * y) + 10 * np.pi * c10 * sy
    u_y = 5 * e * np.cos(5 * y) + np.pi * s10 * cy
    return u_xx + u_yy - np.cos(5 * y) * u_x + np.sin(5 * y) * u_y


def poly5(pts):
    """u = x^3 y^2 - 2 x y^3 + x^2 - 3 y + 1 and its derivatives in the order
    of TERMS_2D (u_xx, u_xy, u_yy, u_x, u_y, u)."""
    x, y = pts[..., 0], pts[..., 1]
    u = x**3 * y**2 - 2 * x * y**3 + x**2 - 3 * y + 1
    return u, (6 * x * y**2 + 2, 6 * x**2 * y - 6 * y**2, 2 * x**3 - 12 * x * y,
               3 * x**2 * y**2 - 2 * y**3 + 2 * x, 2 * x**3 * y - 6 * x * y**2 - 3, u)


def poly5_problem(pts: np.ndarray, bpts: np.ndarray):
    """Variable-coefficient 2D problem (every term on, a Helmholtz-like
    zeroth-order term) whose exact solution is the degree-5 polynomial poly5:
    returns coefficients, source f = L u at the leaf points, boundary data and
    u at the leaf points.  The discretization reproduces polynomials of degree
    <= p - 3 up to rounding, so this checks a solve of any size."""
    c = coeffs_general2d(pts, {
        "xx": lambda x, y: -(1.0 + 0.2 * np.sin(x + 2 * y)),
        "xy": lambda x, y: 0.1 * np.cos(x * y),
        "yy": lambda x, y: -(1.0 + 0.2 * np.cos(x - y)),
        "x": lambda x, y: 0.3 * np.cos(3 * y),
        "y": lambda x, y: -0.2 * np.sin(2 * x),
        "0": lambda x, y: -4.0 * (1.0 + 0.3 * np.sin(3 * x) * np.cos(y)) - 0.5,
    })
    u, d = poly5(pts)
    f = c[:, 0, :] * d[0]
    for t in range(1, 6):
        f += c[:, t, :] * d[t]
    return c, f, poly5(bpts)[0], u


def iti_problem(pts: np.ndarray, bpts: np.ndarray, lo: float = -1.0, hi: float = 1.0):
    """The paper's ItI test problem (Section 5.1, eq. ItI_problem):
    Laplace u + (1 + e^{-50 |x|^2}) u = f on [-1, 1]^2 with Robin data
    u_n + i u = g, manufactured from u = e^{20 i x} + e^{30 i y}.  Returns
    real coefficients [leaf, term, point], complex f at the leaf points,
    complex g at the root boundary points (outward normal of each point's
    side) and u at the leaf points."""
    x, y = pts[..., 0], pts[..., 1]
    c = coeffs_general2d(pts, {"xx": lambda x, y: np.ones_like(x), "yy": lambda x, y: np.ones_like(x),
                               "0": lambda x, y: 1.0 + np.exp(-50 * (x ** 2 + y ** 2))})
    u = np.exp(20j * x) + np.exp(30j * y)
    f = -400 * np.exp(20j * x) - 900 * np.exp(30j * y) + c[:, _term(2, "0"), :] * u
    bx, by = bpts[:, 0], bpts[:, 1]
    ub = np.exp(20j * bx) + np.exp(30j * by)
    ux, uy = 20j * np.exp(20j * bx), 30j * np.exp(30j * by)
    un = np.where(np.isclose(by, lo), -uy, np.where(np.isclose(bx, hi), ux, np.where(np.isclose(by, hi), uy, -ux)))
    return c, f, un + 1j * ub, u


# --------------------------------------------------------------------------
# Per-workload bundles
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# Adaptive 3D workload (the paper's wavefront problem, Section 5: Poisson on
# [0, 1]^3 with u = arctan(10 |x - c| - 0.7)).  Its printed centre (1/2, 1/2,
# 1/2) is a point of every uniform and adaptive grid, where the source has a
# 1/r singularity; the centre here sits slightly off the dyadic grid.
# --------------------------------------------------------------------------
WAVEFRONT_CENTER = (0.5 + 0.0137, 0.5 - 0.0091, 0.5 + 0.0053)


def wavefront_u(pts: np.ndarray, center=WAVEFRONT_CENTER) -> np.ndarray:
    r = np.sqrt(np.sum((pts - np.asarray(center)) ** 2, axis=-1))
    return np.arctan(10.0 * r - 0.7)


def wavefront_f(pts: np.ndarray, center=WAVEFRONT_CENTER) -> np.ndarray:
    """-Laplace u (the operator of coeffs_poisson): u'' + (2 / r) u' with
    t = 10 r - 0.7, u' = 10 / (1 + t^2), u'' = -200 t / (1 + t^2)^2."""
    r = np.sqrt(np.sum((pts - np.asarray(center)) ** 2, axis=-1))
    t = 10.0 * r - 0.7
    d1 = 10.0 / (1.0 + t * t)
    d2 = -200.0 * t / (1.0 + t * t) ** 2
    return -(d2 + 2.0 * d1 / r)


WORKLOADS = {
    1: dict(dim=2, depth=2, p=8, name="poisson2d_L2_p8"),
    2: dict(dim=2, depth=6, p=16, k=40.0, nrhs=16, name="helmholtz2d_k40_L6_p16"),
    3: dict(dim=3, depth=3, p=12, name="divgrad3d_L3_p12"),
    5: dict(dim=2, depth=5, p=16, k=20.0, nfields=32, name="helmholtz2d_k20_L5_p16_grad"),
}

SERVING_OPS = [  # (depth, p, k) of the eight resident serving operators
    (4, 12, 10.0), (4, 16, 20.0), (5, 12, 20.0), (5, 16, 40.0),
    (6, 12, 40.0), (6, 16, 10.0), (7, 12, 20.0), (7, 16, 40.0),
]


def helmholtz_inputs(leaf_pts: np.ndarray, bdry_pts: np.ndarray, k: float,
                     nrhs: int, config: int = 2, op_seed: int = 0):
    """Helmholtz workload: coefficients from 8 seeded bumps and ``nrhs``
    right-hand sides (Fourier boundary data + one source bump each).

    Returns (coeffs [nl, 6, np], bdry [nrhs, nb], src [nrhs, nl, np])."""
    g = rng(config, 100 + op_seed)
    qp = draw_bumps(g, nbumps=8, amp=(0.0, 0.5), box=0.75, dim=2)
    q = eval_bumps(qp, leaf_pts, width=0.1)
    coeffs = coeffs_helmholtz(leaf_pts, k, q)
    bdry = np.empty((nrhs, bdry_pts.shape[0]))
    src = np.empty((nrhs,) + leaf_pts.shape[:-1])
    for r in range(nrhs):
        gr = rng(config, 1000 + 64 * op_seed + r)
        bdry[r] = eval_fourier(draw_fourier(gr), bdry_pts)
        src[r] = eval_bumps(draw_source_bump(gr), leaf_pts, width=0.1)
    return coeffs, bdry, src


def differentiation_inputs(leaf_pts: np.ndarray, bdry_pts: np.ndarray, k: float = 20.0,
                           nfields: int = 32, nobs: int = 256, config: int = 5):
    """Misfit-gradient workload: ``nfields`` seeded scattering potentials q
    (8 bumps each, as the Helmholtz workload), a separately seeded q* whose
    solution supplies the observations, ``nobs`` observation points
    ~ U([-0.9, 0.9]^2), and one right-hand side (Fourier boundary data + one
    source bump).

    Returns dict(q [nfields, nl, np], q_star [nl, np], x_obs [nobs, 2],
    bdry [1, nb], src [1, nl, np], k)."""
    q = np.empty((nfields,) + leaf_pts.shape[:-1])
    for f in range(nfields):
        qp = draw_bumps(rng(config, 200 + f), nbumps=8, amp=(0.0, 0.5), box=0.75, dim=2)
        q[f] = eval_bumps(qp, leaf_pts, width=0.1)
    qs = draw_bumps(rng(config, 199), nbumps=8, amp=(0.0, 0.5), box=0.75, dim=2)
    x_obs = rng(config, 198).uniform(-0.9, 0.9, size=(nobs, 2))
    gr = rng(config, 1000)
    bdry = eval_fourier(draw_fourier(gr), bdry_pts)[None]
    src = eval_bumps(draw_source_bump(gr), leaf_pts, width=0.1)[None]
    return dict(q=q, q_star=eval_bumps(qs, leaf_pts, width=0.1), x_obs=x_obs,
                bdry=bdry, src=src, k=float(k))



def serving_request_params(i: int, config: int = 4):
    """Right-hand side of serving request i: its own seeded Fourier boundary
    series (16 modes, as the Helmholtz workload) and one Gaussian source
    bump (centre ~ U([-0.75, 0.75]^2), amplitude ~ N(0, 1), width 0.1)."""
    g = rng(config, 5000 + i)
    return draw_fourier(g), draw_source_bump(g)


def serving_arrivals(n: int = 4096, rate: float = 2000.0, nops: int = 8, pool: int = 8,
                     config: int = 4):
    """Open-loop request stream: exponential inter-arrival times at ``rate``
    per second, target operator uniform over ``nops``, and which of the
    operator's ``pool`` seeded right-hand sides the request carries.

    Returns (t_arrival [n] seconds, op [n], rhs [n])."""
    g = rng(config, 7)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    ops = g.integers(0, nops, size=n)
    rhs = g.integers(0, pool, size=n)
    return t, ops, rhs
