"""Host bookkeeping: step dimensions and algorithmic flop/byte counts of the
HOTRG step (used for TFLOP/s and roofline figures; no arithmetic on tensors).

Per directional step with left/right dimension dx, up/down dimension dy and
new dimension D' = min(d_cut, dx^2) the contractions cost, in multiply-adds:
  environment halves  2 dx^3 dy^3      (two Gram products, full squares)
  environment combine dx^4 dy^2
  C1                  dx^3 dy^2 D'
  C2                  D' dx^3 dy^3     (dominant, O(D^7))
  C3                  D'^2 dx^2 dy^2
A flop is two per multiply-add; the eigensolver is not counted.
"""


def dims_schedule(d0, d_cut, n_steps):
    out = []
    dx = dy = d0
    for _ in range(n_steps):
        dn = min(d_cut, dx * dx)
        out.append((dx, dy, dn))
        dx, dy = dy, dn
    return out


def step_flops(dx, dy, dn):
    parts = {
        "gram": 2 * 2 * dx**3 * dy**3,
        "combine": 2 * dx**4 * dy**2,
        "c1": 2 * dx**3 * dy**2 * dn,
        "c2": 2 * dn * dx**3 * dy**3,
        "c3": 2 * dn**2 * dx**2 * dy**2,
    }
    parts["total"] = sum(parts.values())
    return parts


def run_flops(d0, d_cut, n_steps):
    return sum(step_flops(*d)["total"] for d in dims_schedule(d0, d_cut, n_steps))


def c2_bytes(dx, dy, dn, elem=8):
    """Algorithmic HBM bytes of the dominant contraction C2: read X1
    (dn dx^2 dy^2) and T (dx^2 dy^2) once, write X2 (dn dx^2 dy^2) once."""
    x = dn * dx * dx * dy * dy
    return elem * (2 * x + dx * dx * dy * dy)
