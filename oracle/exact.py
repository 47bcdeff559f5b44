"""Exact-rational brute force of the stencil loop nests (test infrastructure).

Pure-Python loops over fractions.Fraction, for tiny grids only (8x8, 8^3).
Each value is the exact rational result of the mathematical update, with no
rounding.  When the inputs are small integers and the coefficients dyadic,
every intermediate value of the FP64 computation is representable, so the
FP64 result must equal this exactly; otherwise the difference is bounded by
the rounding analysis stated in the tests.
"""
from fractions import Fraction


def jacobi2d(grid, steps):
    """grid: list of lists (ny x nx) of numbers; boundary held fixed."""
    a = [[Fraction(v) for v in row] for row in grid]
    ny, nx = len(a), len(a[0])
    q = Fraction(1, 4)
    for _ in range(steps):
        b = [row[:] for row in a]
        for i in range(1, ny - 1):
            for j in range(1, nx - 1):
                b[i][j] = q * (a[i - 1][j] + a[i + 1][j] + a[i][j - 1] + a[i][j + 1])
        a = b
    return a


def heat3d(field, steps, alpha):
    """field: nested lists [z][y][x]; alpha: number (converted exactly).
    Returns (final field, list of exact residuals sum (u'-u)^2)."""
    al = Fraction(alpha)
    u = [[[Fraction(v) for v in row] for row in plane] for plane in field]
    nz, ny, nx = len(u), len(u[0]), len(u[0][0])
    residuals = []
    for _ in range(steps):
        w = [[row[:] for row in plane] for plane in u]
        r = Fraction(0)
        for z in range(1, nz - 1):
            for y in range(1, ny - 1):
                for x in range(1, nx - 1):
                    c = u[z][y][x]
                    lap = (u[z][y][x - 1] + u[z][y][x + 1] + u[z][y - 1][x] + u[z][y + 1][x]
                           + u[z - 1][y][x] + u[z + 1][y][x] - 6 * c)
                    w[z][y][x] = c + al * lap
                    r += (w[z][y][x] - c) ** 2
        residuals.append(r)
        u = w
    return u, residuals


def residual_of_stored(u_old, u_new):
    """Exact sum over the interior of (u_new - u_old)^2 for given FP64 arrays
    (numpy), each stored value taken exactly."""
    nz, ny, nx = u_old.shape
    r = Fraction(0)
    for z in range(1, nz - 1):
        for y in range(1, ny - 1):
            for x in range(1, nx - 1):
                d = Fraction(float(u_new[z, y, x])) - Fraction(float(u_old[z, y, x]))
                r += d * d
    return r
