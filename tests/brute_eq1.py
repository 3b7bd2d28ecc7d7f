"""Brute-force evaluation of the paper's Eq. 1 in 50-digit arithmetic (mpmath).

Used only to pin the oracle on tiny inputs. It follows the equation literally:
for every sample i the transmittance T_i is rebuilt from the explicit sum of
sigma_j delta_j over the samples before i (no running product, no log-space
state), the sample's voxel is found by testing every voxel's cell bounds, and
the nearest direction cell by testing every (theta, phi) cell's bounds. The
camera inverse is mpmath's matrix inverse. The bilinear direction lookup
finds the four surrounding cell centres by search and blends them with weights
from the distances to them.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50


def _cell_of(value, lo, hi, n, tie=0):
    """Index of the cell containing value, by search over the cells
    [lo + (i - tie) h, lo + (i + 1 - tie) h) (the first and last cells extend to
    the box faces); None outside [lo, hi]."""
    h = (hi - lo) / n
    if value < lo or value > hi:
        return None
    for i in range(n):
        a = lo if i == 0 else lo + (i - tie) * h
        b = hi if i == n - 1 else lo + (i + 1 - tie) * h
        if a <= value < b or (i == n - 1 and value == b):
            return i
    return None


def _bilinear_beta(beta, l, D, theta, phi):
    """Bilinear blend of the direction cache between the four cell centres
    around (theta, phi), found by searching the centres (theta_j = (j + 1/2)
    pi / l, phi_m = (m + 1/2) 2 pi / l). Below the first or above the last
    theta centre both rows are the edge row; phi wraps around (the centre
    before phi_0 is phi_{l-1} - 2 pi)."""
    th_c = [(j + mp.mpf(1) / 2) * mp.pi / l for j in range(l)]
    ph_c = [(m + mp.mpf(1) / 2) * 2 * mp.pi / l for m in range(l)]
    if theta <= th_c[0]:
        j0 = j1 = 0
        a = mp.mpf(0)
    elif theta >= th_c[-1]:
        j0 = j1 = l - 1
        a = mp.mpf(0)
    else:
        j0 = max(j for j in range(l) if th_c[j] <= theta)
        j1 = j0 + 1
        a = (theta - th_c[j0]) / (th_c[j1] - th_c[j0])
    if phi < ph_c[0]:
        m0, m1, lo_c, hi_c = l - 1, 0, ph_c[-1] - 2 * mp.pi, ph_c[0]
    elif phi >= ph_c[-1]:
        m0, m1, lo_c, hi_c = l - 1, 0, ph_c[-1], ph_c[0] + 2 * mp.pi
    else:
        m0 = max(m for m in range(l) if ph_c[m] <= phi)
        m1, lo_c, hi_c = m0 + 1, ph_c[m0], ph_c[m0 + 1]
    b = (phi - lo_c) / (hi_c - lo_c)

    def cell(j, m):
        return [mp.mpf(float(beta[j][m][c])) for c in range(D)]

    c00, c01, c10, c11 = cell(j0, m0), cell(j0, m1), cell(j1, m0), cell(j1, m1)
    return [(1 - a) * (1 - b) * c00[c] + (1 - a) * b * c01[c] + a * (1 - b) * c10[c] +
            a * b * c11[c] for c in range(D)]


def render_pixel(sigma, u, beta, k, D, l, K, c2w, x, y, near, far, N, eps, bg,
                 bbox=(-1, 1), in_box=False, dir_linear=False):
    lo, hi = mp.mpf(bbox[0]), mp.mpf(bbox[1])
    Km = mp.matrix([[mp.mpf(float(K[r][c])) for c in range(3)] for r in range(3)])
    q = mp.inverse(Km) * mp.matrix([mp.mpf(x) + mp.mpf(1) / 2, mp.mpf(y) + mp.mpf(1) / 2, 1])
    R = mp.matrix([[mp.mpf(float(c2w[r][c])) for c in range(3)] for r in range(3)])
    w = R * q
    n = mp.sqrt(w[0] ** 2 + w[1] ** 2 + w[2] ** 2)
    d = [w[i] / n for i in range(3)]
    o = [mp.mpf(float(c2w[i][3])) for i in range(3)]
    t0, t1 = mp.mpf(near), mp.mpf(far)
    if in_box:
        for a in range(3):
            if d[a] == 0:
                if o[a] < lo or o[a] > hi:
                    return [mp.mpf(b) for b in bg] + [mp.mpf(0)]
                continue
            ta, tb = (lo - o[a]) / d[a], (hi - o[a]) / d[a]
            t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
        if t1 <= t0:
            return [mp.mpf(b) for b in bg] + [mp.mpf(0)]
    delta = (t1 - t0) / N
    theta = mp.acos(max(-1, min(1, d[2])))
    phi = mp.atan2(d[1], d[0])
    if phi < 0:
        phi += 2 * mp.pi
    if dir_linear:
        b = _bilinear_beta(beta, l, D, theta, phi)
    else:
        jt = _cell_of(theta, mp.mpf(0), mp.pi, l)
        mphi = _cell_of(phi, mp.mpf(0), 2 * mp.pi, l) % l
        b = [mp.mpf(float(beta[jt][mphi][c])) for c in range(D)]
    sig, col = [], []
    for i in range(N):
        t = t0 + (i + mp.mpf(1) / 2) * delta
        p = [o[a] + t * d[a] for a in range(3)]
        cells = [_cell_of(p[a], lo, hi, k) for a in range(3)]
        if any(c is None for c in cells):
            sig.append(mp.mpf(0))
            col.append([mp.mpf(0)] * 3)
            continue
        cx, cy, cz = cells
        sig.append(mp.mpf(float(sigma[cz][cy][cx])))
        col.append([mp.fsum(b[c] * mp.mpf(float(u[cz][cy][cx][c][ch])) for c in range(D))
                    for ch in range(3)])
    lim = mp.log(1 / mp.mpf(eps)) if eps > 0 else mp.inf
    C = [mp.mpf(0)] * 3
    T_end = mp.mpf(1)
    for i in range(N):
        Ti = mp.exp(-mp.fsum(sig[j] * delta for j in range(i)))
        if eps > 0 and -mp.log(Ti) > lim:
            T_end = Ti
            break
        a = 1 - mp.exp(-sig[i] * delta)
        for ch in range(3):
            C[ch] += Ti * a * col[i][ch]
    else:
        T_end = mp.exp(-mp.fsum(sig[j] * delta for j in range(N)))
    return [C[ch] + T_end * bg[ch] for ch in range(3)] + [1 - T_end]
