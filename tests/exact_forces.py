"""Exact-rational brute force of the interaction forces (Eqs. 8, 9 and the body force).

An independent third implementation used to pin the oracle: every sum is
carried out with ``fractions.Fraction`` over an explicit list of the 25
offsets of the 5x5 neighbourhood, so the only rounding is the final
conversion to float.  The pseudopotential values (irrational for rational
densities) are taken as given inputs, converted exactly from float64.
"""
from fractions import Fraction as Fr


def w9(e2):
    # D2Q9 weights of the paper (Sec. II A)
    return {0: Fr(4, 9), 1: Fr(1, 9), 2: Fr(1, 36)}.get(e2, Fr(0))


def p25(e2):
    # D2Q25 weights of the paper (Sec. II B)
    return {0: Fr(247, 420), 1: Fr(4, 63), 2: Fr(4, 135), 4: Fr(1, 180),
            5: Fr(2, 945), 8: Fr(1, 15120)}.get(e2, Fr(0))


OFFSETS = [(dx, dy) for dy in range(-2, 3) for dx in range(-2, 3)]


def forces_exact(nx, ny, rho, psi, G1, G2, G_AB, g=((0, 0), (0, 0)), walls=False,
                 rho_wall=(0, 0), psi_wall=(0, 0)):
    """rho, psi: nested lists [k][y][x] of Fractions.  Returns F[k][d][y][x] (Fractions)."""
    def val(arr, wall, k, x, y):
        x %= nx
        if walls and (y < 0 or y >= ny):
            return wall[k]
        return arr[k][y % ny][x]

    F = [[[[Fr(0)] * nx for _ in range(ny)] for _ in range(2)] for _ in range(2)]
    for k in range(2):
        kb = 1 - k
        for y in range(ny):
            for x in range(nx):
                s1 = [Fr(0), Fr(0)]
                s2 = [Fr(0), Fr(0)]
                sr = [Fr(0), Fr(0)]
                for dx, dy in OFFSETS:
                    e2 = dx * dx + dy * dy
                    ps = val(psi, psi_wall, k, x + dx, y + dy)
                    if e2 <= 2:
                        rb = val(rho, rho_wall, kb, x + dx, y + dy)
                        s1[0] += w9(e2) * ps * dx
                        s1[1] += w9(e2) * ps * dy
                        sr[0] += w9(e2) * rb * dx
                        sr[1] += w9(e2) * rb * dy
                    s2[0] += p25(e2) * ps * dx
                    s2[1] += p25(e2) * ps * dy
                for d in range(2):
                    F[k][d][y][x] = (-Fr(G1) * psi[k][y][x] * s1[d]
                                     - Fr(G2) * psi[k][y][x] * s2[d]
                                     - Fr(G_AB) * rho[k][y][x] * sr[d]
                                     + rho[k][y][x] * Fr(g[k][d]))
    return F
