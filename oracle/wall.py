"""Stokeslet and RPY above a no-slip wall (oracle) -- TEST INFRASTRUCTURE ONLY.

The image method of the paper's no-slip wall section (Sec. III, tab:rpywall):
the flow above the plane x_3 = z_w is a sum of free-space summations over
the sources y and their mirror images y^I = (y_1, y_2, 2 z_w - y_3), each
evaluated here by the FP64 direct sums of ``direct``, then assembled at every
target x.  Heights are measured from the wall: h = y_3 - z_w, x_3 = x_3 - z_w.
Per source (f, radius b; b = 0 for the Stokeslet):

  summation  kernel              at y                      at y^I
  S          RPY / Stokeslet     (f_1, f_2, 0), b          (-f_1, -f_2, 0), b
  SD         Laplace q + d       q = -f_3 / 2              q = f_3 / 2, d = h (-f_1, -f_2, f_3)
  SDZ        Laplace q + d       q = h f_3 / 2,            q = -h f_3 / 2,
                                 d = (b^2/6) (0, 0, f_3)   d = (b^2/6) (0, 0, f_3)
  Q          Laplace quadrupole  --                        (b^2/3) [[f_3,0,0],[0,f_3,0],[f_1,f_2,0]]

  u      = u^S + grad phi^SDZ + x_3 grad(phi^SD + phi^Q) - e_3 (phi^SD + phi^Q)
  lap u  = lap u^S + 2 d_3 grad(phi^SD + phi^Q)

Laplace sums use L = 1/(4 pi r), Stokes sums 1/(8 pi) (viscosity 1).

Readings (the table's entries with the kernels normalised as above):
* SD charges.  The table gives q = f_3 at y and -f_3 at y^I.  Writing the
  free-space Stokeslet of a normal force as -e_3 B + x_3 grad B + grad A
  (r_3 r/r^3 = -(x_3 - h) grad(1/r)) fixes B's charge at y to -f_3/2 and
  A's (SDZ) to h f_3 / 2, as the table has for SDZ; the image charge +f_3/2
  and the image dipole h f_3 e_3 then make u vanish on the wall.  With
  (f_3, -f_3) the flow still vanishes on the wall (that pair adds a flow
  -e_3 phi + x_3 grad phi with phi = 0 on the wall) but its singularity at
  y is not the Stokeslet's; the free-space-limit and reciprocity pins fail
  for it and hold for (-f_3/2, f_3/2).
* Quadrupole position.  The table lists the quadrupole under the source
  column.  Applying the source-side RPY operator (1 + b^2/6 lap_y) to the
  b = 0 image system, the only source strength that depends on y is the
  image dipole h (-f_1, -f_2, f_3); lap_y of h D(x - y^I) leaves 2 d/dx_3 of
  that dipole field, a quadrupole at the image.  The quadrupole therefore
  sits at y^I: the no-slip pin fails by ~1e-3 with it at y and holds to
  round-off at y^I.
"""
import numpy as np

from . import direct


def _images(y, zw):
    yi = np.array(y, dtype=np.float64, copy=True)
    yi[:, 2] = 2.0 * zw - yi[:, 2]
    return yi


def _hess_col3(H):
    # (phi, grad, xx, xy, xz, yy, yz, zz) -> d_3 grad phi = (xz, yz, zz)
    return np.stack([H[:, 6], H[:, 8], H[:, 9]], axis=1)


def rpy_wall(y, fb, x, zw=0.0):
    """RPY above the wall: sources y [n,3], (f, b) [n,4] -> (u, lap u) [m,6]."""
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    fb = np.asarray(fb, dtype=np.float64).reshape(-1, 4)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    n = len(y)
    if n == 0:
        return np.zeros((len(x), 6))
    f, b = fb[:, :3], fb[:, 3]
    h = y[:, 2] - zw
    yi = _images(y, zw)
    y2 = np.concatenate([y, yi])
    zero = np.zeros(n)
    # S: RPY of the wall-parallel force and its negated image
    vs = np.concatenate([np.stack([f[:, 0], f[:, 1], zero, b], 1),
                         np.stack([-f[:, 0], -f[:, 1], zero, b], 1)])
    S = direct.rpy(y2, vs, x)
    # SD: charges -f_3/2 and f_3/2, image dipoles h (-f_1, -f_2, f_3)
    SD = direct.laplace(y2, np.concatenate([-0.5 * f[:, 2], 0.5 * f[:, 2]]), yi,
                        h[:, None] * np.stack([-f[:, 0], -f[:, 1], f[:, 2]], 1), x, hess=True)
    # SDZ: charges +-h f_3 / 2, dipoles (b^2/6) (0, 0, f_3) at the source and the image
    dz = np.stack([zero, zero, b * b / 6.0 * f[:, 2]], 1)
    SDZ = direct.laplace(y2, np.concatenate([0.5 * h * f[:, 2], -0.5 * h * f[:, 2]]), y2,
                         np.concatenate([dz, dz]), x)
    # Q: image quadrupoles (b^2/3) [[f_3,0,0],[0,f_3,0],[f_1,f_2,0]]
    Q = np.zeros((n, 3, 3))
    Q[:, 0, 0] = f[:, 2]
    Q[:, 1, 1] = f[:, 2]
    Q[:, 2, 0] = f[:, 0]
    Q[:, 2, 1] = f[:, 1]
    Q *= (b * b / 3.0)[:, None, None]
    QP = direct.laplace_quad(yi, Q.reshape(n, 9), x)
    x3 = (x[:, 2] - zw)[:, None]
    u = S[:, :3] + SDZ[:, 1:4] + x3 * (SD[:, 1:4] + QP[:, 1:4])
    u[:, 2] -= SD[:, 0] + QP[:, 0]
    lap = S[:, 3:] + 2.0 * (_hess_col3(SD) + _hess_col3(QP))
    return np.concatenate([u, lap], axis=1)


def stokeslet_wall(y, f, x, zw=0.0):
    """Stokeslet above the wall: sources y [n,3], f [n,3] -> u [m,3] (the b = 0 system:
    no quadrupole and no SDZ dipoles)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(-1, 3)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    n = len(y)
    if n == 0:
        return np.zeros((len(x), 3))
    h = y[:, 2] - zw
    yi = _images(y, zw)
    y2 = np.concatenate([y, yi])
    zero = np.zeros(n)
    S = direct.stokeslet(y2, np.concatenate([np.stack([f[:, 0], f[:, 1], zero], 1),
                                             np.stack([-f[:, 0], -f[:, 1], zero], 1)]), x)
    SD = direct.laplace(y2, np.concatenate([-0.5 * f[:, 2], 0.5 * f[:, 2]]), yi,
                        h[:, None] * np.stack([-f[:, 0], -f[:, 1], f[:, 2]], 1), x)
    SDZ = direct.laplace(y2, np.concatenate([0.5 * h * f[:, 2], -0.5 * h * f[:, 2]]), None, None, x)
    x3 = (x[:, 2] - zw)[:, None]
    u = S + SDZ[:, 1:4] + x3 * SD[:, 1:4]
    u[:, 2] -= SD[:, 0]
    return u
