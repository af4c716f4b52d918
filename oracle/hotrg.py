"""HOTRG coarse-graining, plain FP64 on the CPU (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Follows Sec. 2 of the paper and its Fig. 1: four copies of the site tensor
give the environment M_{ijkl} of a pair of bonds; the leading left singular
vectors of M, reshaped, give the projector U; two site tensors and two
copies of U give the coarse tensor; the same is then done along the
orthogonal direction; the tensor is divided by its largest element and the
logarithms of these factors accumulate ln Z; after the last step the open
legs are traced with periodic boundary conditions.

Conventions (readings of points the paper leaves open):

* Legs of T are (left, up, right, down).  One *directional step* stacks two
  copies vertically, ``first`` above ``second`` (first.down = second.up), and
  fuses the pair of left legs (second.left, first.left) into one leg, which
  the projector truncates to D' = min(d_cut, D_x**2); the right pair is
  fused the same way.  The orthogonal direction is the same step applied to
  the tensor with its legs transposed, (l, u, r, d) -> (u, l, d, r); two
  directional steps therefore make one iteration of the paper, and K
  directional steps cover 2**K sites.
* The normalisation factor is the largest absolute element, taken after
  every directional step (the paper divides by the largest element once per
  iteration; ln Z is the same in exact arithmetic).
* ln Z / N = ln n_0 + sum_k 2**-k ln n_k + 2**-K ln(sum_{i,j} T_K[i,j,i,j]).
* The projector comes from an SVD of M, as in the paper; M is symmetric
  positive semi-definite, so its singular values are its eigenvalues.
* ``trunc="multiplet"``: when the kept block would split a cluster of
  singular values closer than tau * s_1, the cluster is dropped whole and
  U is padded with zero columns to keep D' columns.

Contractions are written pairwise with ``numpy.tensordot`` in the order that
costs O(D^6) for M and O(D^7) for the coarse tensor.  ``numpy.einsum`` is
not used on the four-operand sums: its path search picks an O(D^9) order.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class StepInfo:
    dx: int           # fused-leg dimension before the step (left/right legs)
    dy: int           # other-leg dimension before the step (up/down legs)
    d_new: int        # D' = min(d_cut, dx*dx): dimension of the new fused leg
    log_norm: float   # ln n_k, n_k = max |T_k| before division
    trunc_err: float  # 1 - sum_{m <= D'} s_m / sum_m s_m
    cut_gap: float    # (s_{D'} - s_{D'+1}) / s_1, or -1 when nothing is cut
    lnz_torus: float  # ln Z / N of the 2**k-site torus built so far
    kept: int         # columns of U that are not zero padding
    side: int = 0     # environment the projector came from: 0 left, 1 right


@dataclass
class Result:
    lnz_per_site: float
    steps: list = field(default_factory=list)
    spectra: list = field(default_factory=list)  # per step: s / s_1, descending


def environment(T):
    """M[(i,j),(k,l)] = sum T[j,a,b,e] T[i,e,c,d] T[l,a,b,f] T[k,f,c,d]
    (Sec. 2, first panel of Fig. 1): the environment of the two left legs of
    a vertical pair, i = second.left, j = first.left.

    Pairwise: A[j,e,l,f] = sum_{a,b} T[j,a,b,e] T[l,a,b,f];
              B[i,e,k,f] = sum_{c,d} T[i,e,c,d] T[k,f,c,d];
              M[i,j,k,l] = sum_{e,f} B[i,e,k,f] A[j,e,l,f].
    """
    dx = T.shape[0]
    A = np.tensordot(T, T, axes=([1, 2], [1, 2]))      # (j, e, l, f)
    B = np.tensordot(T, T, axes=([2, 3], [2, 3]))      # (i, e, k, f)
    M = np.tensordot(B, A, axes=([1, 3], [1, 3]))      # (i, k, j, l)
    M = M.transpose(0, 2, 1, 3)                        # (i, j, k, l)
    return M.reshape(dx * dx, dx * dx)


def projector(M, d_cut, trunc="plain", tau=1e-10):
    """Leading left singular vectors of M (Sec. 2, second panel of Fig. 1).

    Returns (U as (dx*dx, D'), singular values descending, D', kept).
    """
    n = M.shape[0]
    Uf, s, _ = np.linalg.svd(M)
    d_new = min(d_cut, n)
    kept = d_new
    if trunc == "multiplet" and d_new < n:
        while kept > 0 and (s[kept - 1] - s[kept]) <= tau * s[0]:
            kept -= 1
    elif trunc not in ("plain", "multiplet"):
        raise ValueError("trunc must be 'plain' or 'multiplet'")
    U = np.zeros((n, d_new))
    U[:, :kept] = Uf[:, :kept]
    return U, s, d_new, kept


def coarse_tensor(T, U3):
    """T~[i,j,k,l] = sum U[a,b,i] T[b,j,d,c] T[a,c,e,l] U[e,d,k]
    (Sec. 2, third panel of Fig. 1): first = T[b,j,d,c] above
    second = T[a,c,e,l]; U[a,b,i] fuses (second.left, first.left) and
    U[e,d,k] fuses (second.right, first.right).

    Pairwise: X1[a,i,j,d,c] = sum_b U[a,b,i] T[b,j,d,c]            O(D^6)
              X2[i,j,d,e,l] = sum_{a,c} X1[a,i,j,d,c] T[a,c,e,l]   O(D^7)
              T~[i,j,l,k]   = sum_{d,e} X2[i,j,d,e,l] U[e,d,k]     O(D^6)
    """
    X1 = np.tensordot(U3, T, axes=([1], [0]))            # (a, i, j, d, c)
    X2 = np.tensordot(X1, T, axes=([0, 4], [0, 1]))      # (i, j, d, e, l)
    Tt = np.tensordot(X2, U3, axes=([2, 3], [1, 0]))     # (i, j, l, k)
    return Tt.transpose(0, 1, 3, 2)                      # (i, j, k, l)


def coarse_tensor_slice(T, U3, i, k):
    """T~[i, :, k, :] of ``coarse_tensor`` for one pair (i, k), at a cost of
    O(D^5): L[a,j,d,c] = sum_b U[a,b,i] T[b,j,d,c],
    R[a,c,l,d] = sum_e T[a,c,e,l] U[e,d,k], T~[i,j,k,l] = sum_{a,c,d} L R.
    Used to check single outputs of large coarse tensors."""
    L = np.tensordot(U3[:, :, i], T, axes=([1], [0]))          # (a, j, d, c)
    R = np.tensordot(T, U3[:, :, k], axes=([2], [0]))          # (a, c, l, d)
    return np.tensordot(L, R, axes=([0, 2, 3], [0, 3, 1]))     # (j, l)


SIDE_MARGIN = 1e-12  # the two-sided choice takes the right side only when it is this much better


def mirror(T):
    """The tensor reflected left-right: legs (l, u, r, d) -> (r, u, l, d).
    The environment of the mirrored tensor is the environment of the
    original pair's two right legs, (second.right, first.right)."""
    return np.ascontiguousarray(T.transpose(2, 1, 0, 3))


def truncation_error(s, kept):
    """1 - (sum of the kept singular values) / (sum of all of them)."""
    return float(1.0 - s[:kept].sum() / s.sum())


def directional_step(T, d_cut, trunc="plain", tau=1e-10, isometry="one"):
    """One directional coarse-graining: environment, projector, coarse
    tensor.  Returns (T~ with legs (l, u, r, d) of the merged pair,
    singular values, D', kept, side).

    ``isometry="one"`` is the paper's choice (Sec. 2): the projector comes
    from the environment of the left pair of legs and truncates both pairs.
    ``isometry="two"`` is the original HOTRG choice: the projectors of the
    left and of the right environment are both formed and the one with the
    smaller truncation error (epsilon_1 vs epsilon_2) is used for both
    pairs.  The right one is taken only when its error is smaller by more
    than SIDE_MARGIN: for tensors symmetric under reflection (Ising, Potts;
    XY up to charge conjugation) the two errors agree up to rounding, and
    the rule then keeps the left projector, as the one-sided method does.
    """
    dx = T.shape[0]
    M = environment(T)
    U, s, d_new, kept = projector(M, d_cut, trunc, tau)
    side = 0
    if isometry == "two":
        Ur, sr, _, kr = projector(environment(mirror(T)), d_cut, trunc, tau)
        if truncation_error(sr, kr) < truncation_error(s, kept) - SIDE_MARGIN:
            U, s, kept, side = Ur, sr, kr, 1
    elif isometry != "one":
        raise ValueError("isometry must be 'one' or 'two'")
    T_new = coarse_tensor(T, U.reshape(dx, dx, d_new))
    return T_new, s, d_new, kept, side


def rotate(T):
    """Exchange the roles of the two lattice directions: legs
    (l, u, r, d) -> (u, l, d, r).  Applying the directional step to the
    rotated tensor coarse-grains along the orthogonal direction."""
    return np.ascontiguousarray(T.transpose(1, 0, 3, 2))


def torus_trace(T):
    """sum_{i,j} T[i,j,i,j]: one tensor closed on itself with periodic
    boundary conditions (Sec. 2)."""
    return float(np.einsum("ijij->", T))


def run(T0, d_cut, n_steps, trunc="plain", tau=1e-10, spec_len=None, isometry="one"):
    """Full HOTRG: K = n_steps directional steps from the initial tensor T0,
    then the periodic trace.  Returns ``Result`` with ln Z per site."""
    if d_cut < 1 or n_steps < 0:
        raise ValueError("d_cut >= 1 and n_steps >= 0 required")
    T = np.array(T0, dtype=np.float64)
    if T.ndim != 4 or T.shape[0] != T.shape[2] or T.shape[1] != T.shape[3]:
        raise ValueError("T0 must have shape (Dx, Dy, Dx, Dy)")
    n0 = np.abs(T).max()
    T = T / n0
    acc = np.log(n0)
    res = Result(lnz_per_site=np.nan)
    for k in range(1, n_steps + 1):
        dx, dy = T.shape[0], T.shape[1]
        Tt, s, d_new, kept, side = directional_step(T, d_cut, trunc, tau, isometry)
        T = rotate(Tt)
        nk = np.abs(T).max()
        T = T / nk
        acc += np.log(nk) * 2.0 ** (-k)
        tr = torus_trace(T)
        lnz_t = acc + 2.0 ** (-k) * np.log(tr) if tr > 0 else np.nan
        gap = (s[d_new - 1] - s[d_new]) / s[0] if d_new < s.size else -1.0
        err = truncation_error(s, kept)
        res.steps.append(StepInfo(dx, dy, d_new, float(np.log(nk)), err,
                                  float(gap), float(lnz_t), kept, side))
        L = s.size if spec_len is None else min(spec_len, s.size)
        res.spectra.append(s[:L] / s[0])
    tr = torus_trace(T)
    if not tr > 0:
        raise FloatingPointError("final trace is not positive")
    res.lnz_per_site = float(acc + 2.0 ** (-n_steps) * np.log(tr))
    return res


def step_flops(dx, dy, d_new):
    """Multiply-add count x 2 of one directional step with the pairwise
    orders above (environment halves, environment combine, three coarse
    contractions); the SVD is not counted."""
    gram = 2 * dx**3 * dy**3 + dx**4 * dy**2
    coarse = dx**3 * dy**2 * d_new + d_new * dx**3 * dy**3 + d_new**2 * dx**2 * dy**2
    return 2 * (gram + coarse)


def dims_schedule(d0, d_cut, n_steps):
    """(dx, dy, d_new) of every directional step for a square initial
    tensor of bond dimension d0 (host bookkeeping, no arithmetic on T)."""
    out = []
    dx, dy = d0, d0
    for _ in range(n_steps):
        d_new = min(d_cut, dx * dx)
        out.append((dx, dy, d_new))
        # after the step the merged tensor is (d_new, dy, d_new, dy); the
        # rotation swaps the roles: next dx = dy, next dy = d_new
        dx, dy = dy, d_new
    return out
