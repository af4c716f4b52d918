"""Internal energy and specific heat by finite differences (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 3.3 obtains the specific heat as the second derivative of ln Z by a
finite-difference method.  Here ln Z/N comes from ``hotrg.run`` at
beta + j h, j = -2 .. 2, and the derivatives use the five-point central
stencils (error O(h^4)):

  f'(beta)  ~ [f(-2) - 8 f(-1) + 8 f(1) - f(2)] / (12 h)
  f''(beta) ~ [-f(-2) + 16 f(-1) - 30 f(0) + 16 f(1) - f(2)] / (12 h^2)

with the internal energy per site u = -f' and the specific heat per site
c = beta^2 f'' (k_B = 1).
"""

from oracle import hotrg


def thermo(tensor_at, beta, h, d_cut, n_steps, trunc="plain", tau=1e-10, isometry="one"):
    """tensor_at(beta) -> initial tensor.  Returns dict(lnz, energy, cv)."""
    f = [hotrg.run(tensor_at(beta + j * h), d_cut, n_steps, trunc, tau,
                   isometry=isometry).lnz_per_site for j in (-2, -1, 0, 1, 2)]
    d1 = (f[0] - 8.0 * f[1] + 8.0 * f[3] - f[4]) / (12.0 * h)
    d2 = (-f[0] + 16.0 * f[1] - 30.0 * f[2] + 16.0 * f[3] - f[4]) / (12.0 * h * h)
    return {"lnz": f[2], "energy": -d1, "cv": beta * beta * d2}
