"""Discrete operators of App. E (Discrete Function Spaces, Operators and Inner
Products) on a periodic nodal grid.

Grid functions are 2-D arrays indexed ``f[j, i]`` with x_i = i h, y_j = j h,
i, j = 0..n-1; axis 1 is x.  Periodic ghost points (App. E, "Boundary
Conditions") are realised by cyclic shifts.  The paper's typos in this
appendix are read as follows: the 5-point Laplacian has the four distinct
neighbours (the printed formula repeats phi_{i-1,j}), and the edge-to-centre
difference d_x is a difference, not a sum.
"""
import numpy as np


def east(f):
    """f_{i+1,j} (periodic)."""
    return np.roll(f, -1, axis=-1)


def west(f):
    """f_{i-1,j} (periodic)."""
    return np.roll(f, 1, axis=-1)


def north(f):
    """f_{i,j+1} (periodic)."""
    return np.roll(f, -1, axis=-2)


def south(f):
    """f_{i,j-1} (periodic)."""
    return np.roll(f, 1, axis=-2)


# --- centre-to-edge operators A_x, D_x, A_y, D_y (App. E, item 1) -----------
# The edge value at i+1/2 is stored at index i.

def Ax(f):
    return 0.5 * (east(f) + f)


def Dx(f, h):
    return (east(f) - f) / h


def Ay(f):
    return 0.5 * (north(f) + f)


def Dy(f, h):
    return (north(f) - f) / h


# --- edge-to-centre differences d_x, d_y (App. E, item 1) -------------------

def dx_edge(fe, h):
    """d_x f_{ij} = (f_{i+1/2,j} - f_{i-1/2,j}) / h for f stored at i+1/2."""
    return (fe - west(fe)) / h


def dy_edge(fe, h):
    return (fe - south(fe)) / h


# --- centred gradient, divergence, curl, Laplacian (App. E, items 2-4) ------

def grad_x(f, h):
    """x-part of nabla_h: mean of the two adjacent edge differences."""
    dxe = Dx(f, h)
    return 0.5 * (dxe + west(dxe))


def grad_y(f, h):
    dye = Dy(f, h)
    return 0.5 * (dye + south(dye))


def div(u, v, h):
    """nabla_h . (u, v) (App. E, item 3)."""
    return grad_x(u, h) + grad_y(v, h)


def curl(u, v, h):
    """omega = nabla_h x (u, v), the scalar z-component (Eq. discrete_d,
    written out in App. G as Eq. MG_DFT_d)."""
    return grad_x(v, h) - grad_y(u, h)


def lap(f, h):
    """Delta_h f = d_x(D_x f) + d_y(D_y f) (App. E, item 4)."""
    return dx_edge(Dx(f, h), h) + dy_edge(Dy(f, h), h)


# --- inner products and norms (App. E, "Discrete Norms") --------------------

def ip(a, b, h):
    """(a || b) = h^2 sum a b (a NumPy scalar: float64 for real grid functions,
    complex128 for the complex-step derivative checks of the energies)."""
    return h * h * np.sum(np.asarray(a) * np.asarray(b))


def norm2(a, h):
    return np.sqrt(ip(a, a, h))
