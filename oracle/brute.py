"""Brute-force double sum in pure Python (test oracle, tiny inputs only).

A second, independent implementation of the pair part of Eq. (2) of Lazic
et al. (arXiv:0810.2273) with the interpolated Dion kernel, written with
the math module and Python loops only.  It exists to pin the C oracle's
row sums on grids of a few hundred points.  Test infrastructure.
"""
import math


def _phi_tilde(qi, qj, r, tab, n_D, n_sigma, D_max, C):
    D = 0.5 * (qi + qj) * r
    if D >= D_max:
        d1 = qi * r
        d2 = qj * r
        return -C / (d1 ** 2 * d2 ** 2 * (d1 ** 2 + d2 ** 2))
    delta = (qi - qj) / (qi + qj)
    sigma = delta * delta
    step = D_max / (n_D - 1)
    k = min(int(math.floor(D / step)), n_D - 2)
    fD = D / step - k
    l = min(int(math.floor(sigma * (n_sigma - 1))), n_sigma - 2)
    fS = sigma * (n_sigma - 1) - l
    low = tab[k][l] + fS * (tab[k][l + 1] - tab[k][l])
    high = tab[k + 1][l] + fS * (tab[k + 1][l + 1] - tab[k + 1][l])
    return low + fD * (high - low)


def pair_energy(points, h, cell_n, periodic, image_max, r_cut, tab, D_max, dV):
    """points: list of (ix, iy, iz, n, q).  Returns (E over the 0th cell, E over images),
    each 1/2 dV^2 sum n_i n_j phi~, with (i, i, 0) excluded."""
    n_D = len(tab)
    n_sigma = len(tab[0])
    C = 12.0 * (4.0 * math.pi / 9.0) ** 3
    ranges = [range(-image_max[a], image_max[a] + 1) if periodic[a] else range(0, 1) for a in range(3)]
    e_home = 0.0
    e_img = 0.0
    for i, (xi, yi, zi, ni, qi) in enumerate(points):
        for m in ranges[0]:
            for p in ranges[1]:
                for s in ranges[2]:
                    home = (m, p, s) == (0, 0, 0)
                    for j, (xj, yj, zj, nj, qj) in enumerate(points):
                        if home and i == j:
                            continue
                        dx = (xi - xj - m * cell_n[0]) * h[0]
                        dy = (yi - yj - p * cell_n[1]) * h[1]
                        dz = (zi - zj - s * cell_n[2]) * h[2]
                        r = math.sqrt(dx * dx + dy * dy + dz * dz)
                        if r_cut > 0 and r > r_cut:
                            continue
                        v = ni * nj * _phi_tilde(qi, qj, r, tab, n_D, n_sigma, D_max, C)
                        if home:
                            e_home += v
                        else:
                            e_img += v
    return 0.5 * dV * dV * e_home, 0.5 * dV * dV * e_img
