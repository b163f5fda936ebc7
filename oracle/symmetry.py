"""Spinor symmetry unfolding, written out from its definitions.  TEST INFRASTRUCTURE ONLY.

Sec. III (symmetries without spin, with spinor wavefunctions, axis and angle
extraction) of arXiv:2206.00808.  Conventions:

* Orthorhombic cell a = (a1, a2, a3): direct lattice matrix A = diag(a), a
  point r = A x with fractional x; reciprocal vectors G = 2 pi A^-T g with
  integer g.
* An operation {S|tau} maps r to S r + tau.  It is given in the lattice basis:
  integer S_lat acting on fractional coordinates and fractional tau_lat, so
  S_cart = A S_lat A^-1 and G . tau = 2 pi g . tau_lat.
* On reciprocal integer coordinates S acts as S_lat^-T; k' = S_lat^-T k.
* Coefficients c[n][sigma][G] of psi_nk = sum_G c(G) e^{i(k+G).r} chi_sigma.

Function                 | pinned by (tests/test_symmetry_pins.py)
-------------------------|---------------------------------------------------
rotation_lat_to_cart     | A S_lat A^-1 orthogonal for a lattice symmetry;
                         | the reciprocal-basis form (B^T)^-1 S_lat B^T agrees
quaternion_from_rotation | q q^T = X / 4 for random rotations, including
                         | angles at 0 and pi where the trace formula breaks;
                         | rebuilt rotation matrix equals the input
su2_from_rotation        | unitary, det 1, U^H sigma_i U = sum_j R_ij sigma_j
                         | (the spin vector turns with R); improper ops take
                         | the rotation part; q and -q give U and -U
kgrid_orbits             | the orbits partition the grid, every point is its
                         | representative moved by the recorded operation and
                         | G0, the weights sum to the grid size, and chi0 from
                         | the representatives equals the full-grid chi0
chi0_symmetrize          | chi0 from the irreducible points of q's little group,
                         | weighted by their orbits and symmetrised, equals chi0
                         | from states diagonalised at every k of the grid; the
                         | result is invariant under every operation
unfold_spinor            | the unfolded state is an eigenstate of a plane-wave
                         | Hamiltonian with spin-orbit coupling at S k, for
                         | symmorphic and screw operations; chi0 summed over
                         | a full k grid from unfolded states equals the sum
                         | over states diagonalised at every k
"""
from __future__ import annotations

import numpy as np

__all__ = ["rotation_lat_to_cart", "quaternion_from_rotation", "su2_from_rotation",
           "rotate_g", "unfold_spinor", "little_group_shift", "chi0_symmetrize", "kgrid_orbits"]

_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = (_SX, _SY, _SZ)


def rotation_lat_to_cart(s_lat, cell):
    """S_cart = A S_lat A^-1 with A the matrix of lattice vectors as columns
    (Sec. III, the change from the lattice basis to the Cartesian basis)."""
    a = np.diag(np.asarray(cell, dtype=np.float64))
    return a @ np.asarray(s_lat, dtype=np.float64) @ np.linalg.inv(a)


def quaternion_from_rotation(r):
    """Unit quaternion (q1, q2, q3, q4) = (n sin(theta/2), cos(theta/2)) of a proper
    rotation R that turns vectors by theta about n (Sec. III, Markley's variant of
    Shepperd's method).

    Reading: the symmetric 4x4 matrix X is built so that X = 4 q q^T for the
    active rotation R(n, theta) (antisymmetric parts R32 - R23, R13 - R31,
    R21 - R12, which the printed X has for the transposed, attitude form; the
    printed X also repeats R12 where R13 belongs).  The column of largest norm
    gives q up to sign; the sign is fixed so that the chosen component is
    positive (the positive branch).
    """
    r = np.asarray(r, dtype=np.float64)
    t = np.trace(r)
    x = np.array([
        [1 + 2 * r[0, 0] - t, r[0, 1] + r[1, 0], r[0, 2] + r[2, 0], r[2, 1] - r[1, 2]],
        [r[1, 0] + r[0, 1], 1 + 2 * r[1, 1] - t, r[1, 2] + r[2, 1], r[0, 2] - r[2, 0]],
        [r[2, 0] + r[0, 2], r[2, 1] + r[1, 2], 1 + 2 * r[2, 2] - t, r[1, 0] - r[0, 1]],
        [r[2, 1] - r[1, 2], r[0, 2] - r[2, 0], r[1, 0] - r[0, 1], 1 + t]])
    norms = np.linalg.norm(x, axis=0)
    i = int(np.argmax(norms))
    q = x[:, i] / norms[i]
    if q[i] < 0:
        q = -q
    return q


def su2_from_rotation(r_cart):
    """The 2x2 spin rotation of a point operation (Sec. III, spinor wavefunctions).

    An improper operation (det = -1) is inversion times a proper rotation; spin
    is axial, so only the rotation part -S turns it.  From the quaternion, the
    angle theta = 2 atan2(|q_vec|, q4) and axis n = q_vec / |q_vec| give
    U = cos(theta/2) I - i sin(theta/2) n . sigma, the operator that turns a
    spinor's spin vector by R.  Reading: the printed matrix's lower-left entry
    (-n_y + i n_x) sin(theta/2) is not in SU(2) (its determinant is not 1 for
    n_x, n_y not both 0); the form used has (n_y - i n_x) sin(theta/2) there,
    and its overall sign convention is the one under which U^H sigma U turns
    with R (checked against a Hamiltonian with spin-orbit coupling).
    """
    r = np.asarray(r_cart, dtype=np.float64)
    if np.linalg.det(r) < 0:
        r = -r
    q = quaternion_from_rotation(r)
    vn = float(np.sqrt(q[0] ** 2 + q[1] ** 2 + q[2] ** 2))
    if vn == 0.0:
        return np.eye(2, dtype=np.complex128) * np.sign(q[3])
    theta = 2.0 * np.arctan2(vn, q[3])
    n = q[:3] / vn
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return (c * np.eye(2) - 1j * s * (n[0] * _SX + n[1] * _SY + n[2] * _SZ)).astype(np.complex128)


def rotate_g(s_lat, g):
    """Integer reciprocal coordinates of S G: S_lat^-T g (rows of g)."""
    m = np.rint(np.linalg.inv(np.asarray(s_lat, dtype=np.float64)).T).astype(np.int64)
    return np.asarray(g, dtype=np.int64) @ m.T


def unfold_spinor(c, gin, gout, s_lat, tau_lat, cell, g0=(0, 0, 0)):
    """Coefficients at k' = S k - G0 from those at k (Sec. III):
    c'(G') = U c(S^-1 G) e^{-i G.tau} with G = G' - G0 the same plane wave's vector
    relative to S k (k' + G' = S k + G; the common phase e^{-i S k . tau} dropped,
    as in the paper).

    c       complex [nb][nspinor][len(gin)] on the sphere gin at k;
    gout    integer G' of the sphere at k' (any order);
    returns complex [nb][nspinor][len(gout)]; raises if some G' has no preimage.
    For nspinor = 1 the spin rotation is left out.
    """
    c = np.asarray(c, dtype=np.complex128)
    nb, ns, _ = c.shape
    lut = {tuple(g): i for i, g in enumerate(np.asarray(gin, dtype=np.int64).tolist())}
    s_lat = np.asarray(s_lat, dtype=np.int64)
    gq = np.asarray(gout, dtype=np.int64) - np.asarray(g0, dtype=np.int64)[None, :]
    # S^-1 on reciprocal integer coordinates is (S_lat^-T)^-1 = S_lat^T
    src = gq @ s_lat
    idx = np.array([lut.get(tuple(g), -1) for g in src.tolist()], dtype=np.int64)
    if np.any(idx < 0):
        raise ValueError("an output G has no preimage in the input sphere")
    phase = np.exp(-2j * np.pi * (gq @ np.asarray(tau_lat, dtype=np.float64)))
    out = c[:, :, idx] * phase[None, None, :]
    if ns == 2:
        u = su2_from_rotation(rotation_lat_to_cart(s_lat, cell))
        out = np.einsum("st,btg->bsg", u, out)
    return out


def little_group_shift(s_lat, qred):
    """G_S with S q = q + G_S (integer reciprocal coordinates), or None when S is
    not in the little group of q."""
    sq = np.linalg.inv(np.asarray(s_lat, dtype=np.float64)).T @ np.asarray(qred, dtype=np.float64)
    gs = sq - np.asarray(qred, dtype=np.float64)
    r = np.rint(gs)
    return r.astype(np.int64) if np.allclose(gs, r, atol=1e-9) else None


def chi0_symmetrize(chi, geps, ops, qred):
    """Average chi0(q) over the little group of q (Sec. III: sums over k are
    unfolded with the little group of q).

    With the unfolding rule above, the pair (v at S(k+q) - G_S, c at S k) has
    M_{Sk}(G) = e^{i(q+G).tau} M_k(S^-1 (G - G_S)), since S^-1 (q+G) = q + S^-1 (G - G_S)
    and the spinor rotation cancels in conj(psi_v) psi_c.  Hence
      chi0_{Sk}(G, G') = e^{-i(G-G').tau} chi0_k(S^-1 (G - G_S), S^-1 (G' - G_S)),
    and the sum over a full k grid equals (1/|G_q|) sum_S T_S(sum_i w_i chi0_{k_i})
    over irreducible points k_i with orbit sizes w_i.  This function applies
    (1/n) sum_S T_S to chi (complex [..., N, N] on the sphere geps).
    """
    x = np.asarray(chi, dtype=np.complex128)
    g = np.asarray(geps, dtype=np.int64)
    lut = {tuple(v): i for i, v in enumerate(g.tolist())}
    out = np.zeros_like(x)
    for s_lat, tau in ops:
        gs = little_group_shift(s_lat, qred)
        if gs is None:
            raise ValueError("operation not in the little group of q")
        src = (g - gs[None, :]) @ np.asarray(s_lat, dtype=np.int64)  # S^-1 = S_lat^T
        idx = np.array([lut.get(tuple(v), -1) for v in src.tolist()])
        if np.any(idx < 0):
            raise ValueError("the eps sphere is not closed under the operation")
        ph = np.exp(-2j * np.pi * (g @ np.asarray(tau, dtype=np.float64)))
        out += ph[:, None] * np.conj(ph)[None, :] * x[..., idx[:, None], idx[None, :]]
    return out / len(ops)


def kgrid_orbits(n, ops):
    """Orbits of the unshifted grid k = (i1/n1, i2/n2, i3/n3) under the point
    parts of `ops` (Sec. III: the k-sum over the irreducible wedge of the little
    group of q).  Points are indexed (i1 n2 + i2) n3 + i3; the representative of
    an orbit is its first point in that order.  Returns rep[i], op[i] (an
    operation with S k_rep = k_i + G0), g0[i] (that integer G0) and weight[i]
    (orbit size at representatives, 0 elsewhere).
    """
    n = np.asarray(n, dtype=np.int64)
    npts = int(np.prod(n))
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in n], indexing="ij"), -1).reshape(-1, 3)
    k = idx / n[None, :]
    rep = np.full(npts, -1, dtype=np.int64)
    opi = np.zeros(npts, dtype=np.int64)
    g0 = np.zeros((npts, 3), dtype=np.int64)
    weight = np.zeros(npts, dtype=np.int64)
    for i in range(npts):
        if rep[i] >= 0:
            continue
        for j, (s_lat, _) in enumerate(ops):
            sk = np.linalg.inv(np.asarray(s_lat, dtype=np.float64)).T @ k[i]
            cell = np.floor(sk + 1e-9)
            frac = sk - cell
            t = np.rint(frac * n)
            if np.abs(frac * n - t).max() > 1e-6:
                raise ValueError("the grid is not closed under an operation")
            t = np.mod(t, n).astype(np.int64)
            m = int((t[0] * n[1] + t[1]) * n[2] + t[2])
            if rep[m] < 0:
                rep[m], opi[m] = i, j
                g0[m] = np.rint(sk - k[m]).astype(np.int64)
                weight[i] += 1
    return rep, opi, g0, weight
