"""Measurements of whole-run physics shared by the oracle and GPU physics
tests: lens set-up (eq:N35 pattern), contact angles and lens geometry
(Sec. 4.2, eq:N32-N34).  Plain NumPy on fields read back as FP64."""
import numpy as np

import workloads as W


def lens_setup(nx, ny, R, s12, s13, s23, rho=(1.0, 1.0, 1.0), W_=4.0):
    """Phase 1 lens of radius R at the centre of a flat phase-2 (top) /
    phase-3 (bottom) interface (eq:N35), walls in y, tau_g = tau_i = 0.8
    (mu = 0.1 rho), m = 0.1."""
    xc, yc = nx / 2.0, ny / 2.0
    cl = W.disc(nx, ny, xc, yc, R, W_)
    x, y = W.grid(nx, ny)
    ct = np.maximum(0.5 + 0.5 * np.tanh(2.0 * (y - yc) / W_) - cl, 0.0)
    c = np.stack([cl, ct, 1.0 - cl - ct])
    sig = np.array([[0.0, s12, s13], [s12, 0.0, s23], [s13, s23, 0.0]])
    rho = np.asarray(rho, dtype=float)
    return c, dict(N=3, nx=nx, ny=ny, sigma=sig, rho=rho, mu=0.1 * rho, mobility=0.1,
                   tau_phi=0.8, W=W_, wall_y=True)


def flat_level(c):
    """Level of the flat 2|3 interface far from the lens (column x = 0):
    where c_2 crosses 1/2, linearly interpolated."""
    col = c[1][:, 0]
    j = np.where((col[:-1] < 0.5) & (col[1:] >= 0.5))[0][0]
    return j + (0.5 - col[j]) / (col[j + 1] - col[j])


def _arc_points(c1, yf, upper):
    ny, nx = c1.shape
    pts = []
    for x in range(nx):
        v = c1[:, x]
        if v.max() < 0.5:
            continue
        idx = np.where(v >= 0.5)[0]
        if upper:
            q = idx[-1]
            if q + 1 < ny:
                yy = q + (v[q] - 0.5) / (v[q] - v[q + 1])
                if yy > yf + 2:
                    pts.append((x, yy))
        else:
            q = idx[0]
            if q >= 1:
                yy = q - (v[q] - 0.5) / (v[q] - v[q - 1])
                if yy < yf - 2:
                    pts.append((x, yy))
    return np.array(pts)


def lens_angles(c):
    """Contact angles (degrees) of the upper (phase 1|2) and lower (1|3) lens
    arcs against the flat 2|3 interface: least-squares circles through the
    c_1 = 1/2 contour, middle 70% of each arc (away from the diffuse triple
    junctions); the angle is that of the circle where it meets the level of
    the flat interface far from the lens."""
    c1 = c[0]
    yf = flat_level(c)

    def circle(upper):
        P = _arc_points(c1, yf, upper)
        xm, hw = 0.5 * (P[:, 0].min() + P[:, 0].max()), 0.5 * (P[:, 0].max() - P[:, 0].min())
        P = P[np.abs(P[:, 0] - xm) <= 0.7 * hw]
        A = np.stack([P[:, 0], P[:, 1], np.ones(len(P))], 1)
        a, b, cc = np.linalg.lstsq(A, P[:, 0] ** 2 + P[:, 1] ** 2, rcond=None)[0]
        return a / 2, b / 2, np.sqrt(cc + a * a / 4 + b * b / 4)

    _, yu, ru = circle(True)
    _, yl, rl = circle(False)
    return (np.degrees(np.arccos((yf - yu) / ru)), np.degrees(np.arccos((yl - yf) / rl)))


def lens_geometry(c):
    """The paper's lens measures (Sec. 4.2): length d between the triple
    junctions, cap heights h_1 (above the flat interface, into phase 2) and
    h_2 (below, into phase 3), the angles theta_i = 2 atan(2 h_i / d), and
    the lens area A (nodes with c_1 >= 1/2).  On the c_1 = 1/2 contour:
    h_i from the extreme crossings of the columns, d from the crossings of
    the row interpolated to the flat-interface level."""
    c1 = c[0]
    yf = flat_level(c)
    up = _arc_points(c1, yf, True)
    lo = _arc_points(c1, yf, False)
    h1 = up[:, 1].max() - yf
    h2 = yf - lo[:, 1].min()
    j = int(np.floor(yf))
    t = yf - j
    row = (1.0 - t) * c1[j] + t * c1[j + 1]
    inside = np.where(row >= 0.5)[0]
    a, b = inside[0], inside[-1]
    xl = a - (row[a] - 0.5) / (row[a] - row[a - 1])
    xr = b + (row[b] - 0.5) / (row[b] - row[b + 1])
    d = xr - xl
    th = np.degrees(2.0 * np.arctan(2.0 * np.array([h1, h2]) / d))
    return dict(d=d, h1=h1, h2=h2, theta1=th[0], theta2=th[1], A=float((c1 >= 0.5).sum()))


def neumann_angles(s12, s13, s23):
    """Equilibrium contact angles (degrees) from the tensions, eq:N32."""
    t1 = np.degrees(np.arccos((s12 ** 2 + s23 ** 2 - s13 ** 2) / (2 * s12 * s23)))
    t2 = np.degrees(np.arccos((s13 ** 2 + s23 ** 2 - s12 ** 2) / (2 * s13 * s23)))
    return t1, t2


def lens_shape(A, theta1, theta2):
    """Length d and heights h_1, h_2 of a lens of area A with contact
    angles theta_i (degrees): eq:N33 solved for d, then eq:N34."""
    th = np.radians([theta1, theta2])
    s = np.sum((th / np.sin(th) - np.cos(th)) / np.sin(th))
    half = np.sqrt(A / s)
    h = half * (1.0 - np.cos(th)) / np.sin(th)
    return 2.0 * half, h[0], h[1]


def puddle_thickness(c):
    """Largest thickness of the phase-1 puddle over the columns: distance
    between its lower and upper c_1 = 1/2 crossings."""
    c1 = c[0]
    ny, nx = c1.shape
    best = 0.0
    for x in range(nx):
        v = c1[:, x]
        if v.max() < 0.5:
            continue
        idx = np.where(v >= 0.5)[0]
        lo, hi = idx[0], idx[-1]
        if lo < 1 or hi + 1 >= ny:
            continue
        ylo = lo - (v[lo] - 0.5) / (v[lo] - v[lo - 1])
        yhi = hi + (v[hi] - 0.5) / (v[hi] - v[hi + 1])
        best = max(best, yhi - ylo)
    return best


def de_gennes_thickness(s12, s13, s23, rho1, rho2, rho3, g):
    """Asymptotic thickness H of a large puddle of phase 1 floating between a
    lighter phase 2 above and a heavier phase 3 below.  Isostasy fixes the
    parts above and below the far-field level, a (rho_1 - rho_2) = b (rho_3 -
    rho_1), and the excess hydrostatic pressure integrated over the puddle's
    cross-section, g H^2 (rho_1 - rho_2)(rho_3 - rho_1) / (2 (rho_3 -
    rho_2)), balances sigma_12 + sigma_13 - sigma_23.  With rho_2 = 0 this is
    eq:N37."""
    eff = (rho1 - rho2) * (rho3 - rho1) / (rho3 - rho2)
    return np.sqrt(2.0 * (s12 + s13 - s23) / (eff * g))


def centroid_velocity(c, u, k):
    """Velocity of the centroid of phase k: sum c_k u / sum c_k."""
    m = c[k].sum()
    return (c[k] * u[0]).sum() / m, (c[k] * u[1]).sum() / m


def order_parameters(c, rho):
    """phi_i of eq:N12 from the volume fractions (the inverse the initial
    state uses): phi_i = (rho_i c_i - rho_N c_N - b_i) / a_i."""
    rho = np.asarray(rho, dtype=float)
    a = 0.5 * (rho[:-1] + rho[-1])
    b = 0.5 * (rho[:-1] - rho[-1])
    return np.stack([(rho[i] * c[i] - rho[-1] * c[-1] - b[i]) / a[i]
                     for i in range(len(rho) - 1)])


def line_tension(c_line, rho, lam):
    """Tension of an interface crossed by the 1-D profile c_line (N, n),
    taken along its normal: at equilibrium the gradient and bulk parts of
    the free energy are equal (equipartition), so sigma = int sum_ij
    lambda_ij phi_i' phi_j' (central differences, unit spacing)."""
    d = np.gradient(order_parameters(c_line, rho), axis=1)
    return float(np.einsum("ij,in,jn->n", lam, d, d).sum())


def lens_interface_lines(c):
    """Profiles across the three interfaces of an equilibrated lens (phase 1
    lens at the flat interface between phase 2 above and phase 3 below):
    the column far from the lens (x = 0) crosses 2|3, the column through the
    lens centre crosses 1|2 above the flat level and 1|3 below it.  Returns
    {(k, l): (profile, index of the third phase)} with 0-based phases."""
    ny, nx = c.shape[1:]
    yf = int(round(flat_level(c)))
    xc = nx // 2
    return {(1, 2): (c[:, :, 0], 0),
            (0, 1): (c[:, yf + 1:, xc], 2),
            (0, 2): (c[:, :yf, xc], 1)}
