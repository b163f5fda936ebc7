"""Plain CPU FP64 oracle of the spinor Epsilon path.  TEST INFRASTRUCTURE ONLY.

Slow and direct on purpose.  Each function states the passage of the paper
(arXiv:2206.00808, "Fully relativistic GW/Bethe-Salpeter calculations in
BerkeleyGW") it writes out.  Conventions (the readings are listed in the
design notes):

* Hartree energies; cutoffs on |k+G|^2 in bohr^-2 (Rydberg); orthorhombic
  cell a = (a1, a2, a3); G = 2 pi g / a for integer g.
* One k-point (k = 0, N_k = 1 unless a prefactor is passed): occupied (valence)
  states at k+q, empty (conduction) states at k, as in the Adler-Wiser sum of
  Sec. II.
* Coefficients c[n][sigma][G] with sigma = up, down; the periodic part of a
  spinor component on the grid is u(r_j) = sum_G c(G) exp(+2 pi i g.j / n).
* M_vc(G) = sum_sigma <v,k+q,sigma| e^{i(q+G).r} |c,k,sigma>
          = sum_sigma (1/N) sum_j conj(u_v(r_j)) u_c(r_j) exp(+2 pi i g.j / n).

Function                 | pinned by (tests/test_oracle_pins.py)
-------------------------|---------------------------------------------------
wavefunction_on_box      | brute-force synthesis, unit-norm (Parseval)
mtxel_fft                | convolution form, brute force, single plane wave
mtxel_convolution        | brute force, single plane wave, orthonormality
mtxel_bruteforce         | closed forms on single plane waves
chi0                     | scipy ZHERK, Hermitian/NSD, Loewner, asymptote,
                         | doubled collinear set (spinor = 2 x spinless)
chi0_weight_real         | imaginary-axis factor at w = i omega, eta = 0;
                         | the summed form 2a/(a^2 - w^2), a = delta + i eta
chi0_real                | scipy ZHERK on the real and imaginary weight parts,
                         | even in w, absorptive diagonal, static limit
epsilon / epsilon_inverse| Sherman-Morrison closed form, eigenvalue bounds,
                         | LU solve via scipy
head_overlap             | convolution form at G = 0, orthonormality
head_dipole              | k.p limit of head_overlap for a spin-dependent
                         | local-potential model, Hermiticity, plane waves
epsinv_lowrank           | exact inverse at nb = N; rank-one chi0 exact at nb = 1
                         | (Sherman-Morrison); at omega = 0 the error is the
                         | discarded eigenvalues' 1/lambda - 1 (closed form)
epsinv_projected         | equals epsinv_lowrank (chi0 projected after the sum)
                         | for the same basis; exact when chi0's range is nb-dim
screened_w               | Hermitian for the symmetric form of eps (closed form)
sigma_sx_static          | bare exchange at eps^-1 = I (closed form), real and
                         | between the bare exchange and 0 for chi0 <= 0
gpp_modes / epsinv_gpp   | eps^-1_GPP(0) = eps^-1 on kept modes (closed form);
                         | f-sum rule by quadrature of the broadened pole
bse_kernel               | real-space double sums over the grid with the
                         | Coulomb and W kernels built from their Fourier
                         | series; collinear spinors give the spinless kernels
                         | in the same-spin blocks and 0 across spin flips;
                         | K^X Hermitian PSD, D + K^X + K^D Hermitian
sigma_gpp                | SX at E = E_n'' equals sigma_sx_static on the GPP's
                         | static eps^-1; COH from the w' > 0 integral of the
                         | broadened pole by quadrature; static COH limit
                         | 1/2 m^H (eps^-1 - 1) v m for wtilde >> |E - E_n''|
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "box_offsets", "wavefunction_on_box", "mtxel_fft", "mtxel_convolution",
    "mtxel_bruteforce", "chi0_weight", "chi0", "chi0_weight_real", "chi0_real", "epsilon",
    "epsilon_inverse",
    "head_overlap", "head_dipole", "screened_w", "sigma_sx_static", "GPP_DROP_TOL", "gpp_modes",
    "epsinv_gpp", "sigma_gpp", "bse_kernel", "epsinv_lowrank", "epsinv_projected", "chi0_from_system", "rel_f", "alias_free",
]


def box_offsets(g, box):
    """Box index of each integer G: g mod n along every axis."""
    return np.mod(np.asarray(g, dtype=np.int64), np.asarray(box, dtype=np.int64))


def alias_free(gv, gc, geps, box):
    """True when no product component can alias onto an eps-sphere G.

    The product conj(u_v) u_c holds Fourier components g_c - g_v; a component
    folds onto -G of the eps sphere only if |g_c - g_v + G|_i >= n_i, which
    cannot happen when n_i > max|g_v|_i + max|g_c|_i + max|G_eps|_i.
    """
    m = (np.abs(gv).max(0) + np.abs(gc).max(0) + np.abs(geps).max(0))
    return bool(np.all(np.asarray(box) > m))


def _ifftn(a, axes, workers):
    """numpy's inverse FFT, or scipy's with `workers` threads (the same transform)."""
    if workers is None:
        return np.fft.ifftn(a, axes=axes)
    import scipy.fft
    return scipy.fft.ifftn(a, axes=axes, workers=workers)


def wavefunction_on_box(c, g, box, workers=None):
    """Periodic part of every spinor component on the real-space grid.

    Sec. II (matrix elements via FFT): the spinor components phi_{nk,alpha}(r)
    are brought to real space before their product is formed.
    u_n^sigma(r_j) = sum_{G in sphere} c_n^sigma(G) exp(+2 pi i g.j/n), i.e.
    N * numpy.fft.ifftn of the coefficients placed at g mod n.
    c: [nb][ns][ng] complex128 -> [nb][ns][n1][n2][n3] complex128
    """
    c = np.asarray(c, dtype=np.complex128)
    nb, ns, ng = c.shape
    box = tuple(int(x) for x in box)
    field = np.zeros((nb, ns) + box, dtype=np.complex128)
    o = box_offsets(g, box)
    field[:, :, o[:, 0], o[:, 1], o[:, 2]] = c
    return _ifftn(field, (2, 3, 4), workers) * float(np.prod(box))


def mtxel_fft(cv, gv, cc, gc, geps, box, workers=None):
    """M_vc(G) by the route of Eq. (matrix_el): per spin component, the
    inverse-transform of the real-space product, then the sum over spin.

    Sec. II, Eq. (matrix_el) and the M_nn'(k,q,G) definition before it:
    for each spin alpha, rho_alpha(r) = conj(phi_{v,k+q,alpha}(r)) phi_{c,k,alpha}(r)
    is transformed with the exp(+i G.r)/N kernel and only then summed over
    alpha.  Returns M[nv][nc][neps] complex128.  `workers` threads the FFTs
    (scipy.fft) and changes nothing else.
    """
    box = tuple(int(x) for x in box)
    uv = wavefunction_on_box(cv, gv, box, workers)
    uc = wavefunction_on_box(cc, gc, box, workers)
    nv, ns = uv.shape[:2]
    nc = uc.shape[0]
    o = box_offsets(geps, box)
    out = np.zeros((nv, nc, len(geps)), dtype=np.complex128)
    for v in range(nv):
        for c in range(nc):
            acc = np.zeros(len(geps), dtype=np.complex128)
            for s in range(ns):
                rho = np.conj(uv[v, s]) * uc[c, s]
                t = _ifftn(rho, (0, 1, 2), workers)
                acc += t[o[:, 0], o[:, 1], o[:, 2]]
            out[v, c] = acc
    return out


def _shift_index(gsrc_lookup, g_list, shift):
    """Index in a sphere of each g - shift, or -1 if it lies outside."""
    idx = np.empty(len(g_list), dtype=np.int64)
    for i, g in enumerate(g_list):
        idx[i] = gsrc_lookup.get((g[0] - shift[0], g[1] - shift[1], g[2] - shift[2]), -1)
    return idx


def mtxel_convolution(cv, gv, cc, gc, geps):
    """M_vc(G) from its definition written in the plane-wave basis, no grid.

    Sec. II, definition of M_nn'(k,q,G): with phi_{v,k+q} = sum c_v(G1)
    e^{i(k+q+G1).r} and phi_{c,k} = sum c_c(G2) e^{i(k+G2).r}, the cell integral of
    conj(phi_v) e^{i(q+G).r} phi_c keeps only G2 = G1 - G, so
    M_vc(G) = sum_alpha sum_{G1} conj(c_v^alpha(G1)) c_c^alpha(G1 - G).
    Returns M[nv][nc][neps].
    """
    cv = np.asarray(cv, dtype=np.complex128)
    cc = np.asarray(cc, dtype=np.complex128)
    nv, ns, ngv = cv.shape
    nc = cc.shape[0]
    lut = {tuple(g): i for i, g in enumerate(np.asarray(gc).tolist())}
    gvl = np.asarray(gv).tolist()
    out = np.zeros((nv, nc, len(geps)), dtype=np.complex128)
    a = np.conj(cv).reshape(nv, ns * ngv)
    for ig, G in enumerate(np.asarray(geps).tolist()):
        idx = _shift_index(lut, gvl, G)
        ok = idx >= 0
        b = np.zeros((nc, ns, ngv), dtype=np.complex128)
        b[:, :, ok] = cc[:, :, idx[ok]]
        out[:, :, ig] = a @ b.reshape(nc, ns * ngv).T
    return out


def mtxel_bruteforce(cv, gv, cc, gc, geps, box):
    """Explicit real-space sums, no FFT: for tiny grids only.

    Synthesises u(r_j) = sum_G c(G) exp(2 pi i g.j/n) point by point and
    projects M(G) = (1/N) sum_j sum_alpha conj(u_v) u_c exp(2 pi i g.j/n).
    """
    box = np.asarray(box, dtype=np.int64)
    n_total = int(np.prod(box))
    j = np.stack(np.meshgrid(*[np.arange(n) for n in box], indexing="ij"), -1).reshape(-1, 3)
    frac = j / box  # r_j in units of the cell vectors

    def synth(c, g):
        ph = np.exp(2j * np.pi * (frac @ np.asarray(g, dtype=np.float64).T))  # [N, ng]
        return np.einsum("rg,bsg->bsr", ph, np.asarray(c, dtype=np.complex128))

    uv = synth(cv, gv)
    uc = synth(cc, gc)
    proj = np.exp(2j * np.pi * (frac @ np.asarray(geps, dtype=np.float64).T))  # [N, neps]
    rho = np.einsum("vsr,csr->vcr", np.conj(uv), uc)
    return np.einsum("vcr,rg->vcg", rho, proj) / n_total


def chi0_weight(ev, ec, omega):
    """Adler-Wiser energy factor on the imaginary axis, eta = 0.

    Sec. II, polarizability P_GG'(q, w): the bracket
    1/(e_v - e_c - w + i eta) + 1/(e_v - e_c + w + i eta) taken at w -> i*omega
    and eta = 0; both terms are kept as written and summed.
    Returns w[nfreq][nv*nc] (real: the imaginary parts cancel).
    """
    ev = np.asarray(ev, dtype=np.float64)
    ec = np.asarray(ec, dtype=np.float64)
    delta = (ev[:, None] - ec[None, :]).reshape(-1)
    out = []
    for om in np.atleast_1d(np.asarray(omega, dtype=np.float64)):
        w = 1.0 / (delta - 1j * om) + 1.0 / (delta + 1j * om)
        out.append(w.real)
    return np.array(out)


def chi0(mtxel, ev, ec, omega, prefactor=1.0):
    """P_GG'(q, i omega) = (1/N_k) sum_{v,c} M*_vc(G) M_vc(G') [Adler-Wiser bracket].

    Sec. II, the polarizability P_GG'(q, w) at imaginary frequency, one k-point.
    mtxel: [nv][nc][neps].  Returns chi0[nfreq][neps][neps] complex128.
    """
    m = np.asarray(mtxel, dtype=np.complex128)
    nv, nc, neps = m.shape
    flat = m.reshape(nv * nc, neps)
    w = chi0_weight(ev, ec, omega)
    return np.stack([prefactor * ((np.conj(flat).T * wf[None, :]) @ flat) for wf in w])


def chi0_weight_real(ev, ec, omega, eta):
    """Adler-Wiser energy factor with broadening, as Sec. II writes it.

    The bracket 1/(e_v - e_c - w + i eta) + 1/(e_v - e_c + w + i eta) for every
    frequency w of `omega` (real frequencies for the real-axis polarizability;
    a complex w = i*omega' with eta = 0 gives the imaginary-axis factor).
    Returns complex w[nfreq][nv*nc].
    """
    ev = np.asarray(ev, dtype=np.float64)
    ec = np.asarray(ec, dtype=np.float64)
    delta = (ev[:, None] - ec[None, :]).reshape(-1)
    out = []
    for om in np.atleast_1d(np.asarray(omega, dtype=np.complex128)):
        out.append(1.0 / (delta - om + 1j * eta) + 1.0 / (delta + om + 1j * eta))
    return np.array(out)


def chi0_real(mtxel, ev, ec, omega, eta, prefactor=1.0):
    """P_GG'(q, w) on the real frequency axis with broadening eta (Sec. II).

    (1/N_k) sum_{v,c} M*_vc(G) M_vc(G') times the complex bracket of
    chi0_weight_real; the result is not Hermitian.  mtxel: [nv][nc][neps].
    Returns chi0[nfreq][neps][neps] complex128.
    """
    m = np.asarray(mtxel, dtype=np.complex128)
    nv, nc, neps = m.shape
    flat = m.reshape(nv * nc, neps)
    w = chi0_weight_real(ev, ec, omega, eta)
    return np.stack([prefactor * ((np.conj(flat).T * wf[None, :]) @ flat) for wf in w])


def epsilon(chi0_f, vcoul):
    """eps_GG' = delta_GG' - v(q+G) P_GG'  (Sec. II, dielectric matrix)."""
    c = np.asarray(chi0_f, dtype=np.complex128)
    v = np.asarray(vcoul, dtype=np.float64)
    n = c.shape[-1]
    return np.eye(n, dtype=np.complex128) - v[:, None] * c


def epsilon_inverse(chi0_all, vcoul):
    """eps^-1 for every frequency by LAPACK getrf/getri (numpy.linalg.inv).

    Sec. II defines W = eps^-1 v; the Performance section names the inversion
    of the dielectric matrix as a large part of Epsilon's run time.
    """
    c = np.asarray(chi0_all, dtype=np.complex128)
    return np.stack([np.linalg.inv(epsilon(cf, vcoul)) for cf in c])


def epsinv_lowrank(chi0_all, vcoul, nb):
    """eps^-1 in a reduced basis of static eigenvectors (Sec. IV, Bi2Se3: the
    full-frequency calculation keeps 200 eigenvectors, about a tenth of the
    spectrum).  With V = diag(v), epst(w) = I - V^1/2 chi0(w) V^1/2 (Hermitian; eps
    is similar to it), U the eigenvectors of epst(0) with the nb largest
    eigenvalues (numpy.linalg.eigh), and epst_B(w) = U^H epst(w) U:
      epst^-1(w) ~= I + U (epst_B(w)^-1 - I) U^H,   eps^-1 = V^1/2 epst^-1 V^-1/2.
    Outside span(U) the screening is left out (epst^-1 acts as I there).
    Returns (epsinv [nfreq][N][N], eigenvalues of epst(0) in ascending order).
    """
    c = np.asarray(chi0_all, dtype=np.complex128)
    v = np.asarray(vcoul, dtype=np.float64)
    sv = np.sqrt(v)
    n = c.shape[-1]
    epst = np.eye(n)[None] - sv[None, :, None] * c * sv[None, None, :]
    lam, vec = np.linalg.eigh(epst[0])
    u = vec[:, n - nb:]
    out = []
    for e in epst:
        eb = u.conj().T @ e @ u
        et = np.eye(n) + u @ (np.linalg.inv(eb) - np.eye(nb)) @ u.conj().T
        out.append(sv[:, None] * et / sv[None, :])
    return np.stack(out), lam


def epsinv_projected(mtxel, ev, ec, omega, vcoul, u, prefactor=1.0):
    """The same reduced-basis eps^-1 with chi0 built in the basis: with
    M_B = M diag(sqrt v) U, chi_B(w) = sum_p w_p(w) conj(M_B,p) M_B,p^T equals
    U^H V^1/2 chi0(w) V^1/2 U, and
      epst^-1(w) ~= I + U ((I - chi_B(w))^-1 - I) U^H,  eps^-1 = V^1/2 epst^-1 V^-1/2.
    u: [N][nb] orthonormal columns.  Returns [nfreq][N][N]."""
    m = np.asarray(mtxel, dtype=np.complex128)
    nv, nc, n = m.shape
    v = np.asarray(vcoul, dtype=np.float64)
    sv = np.sqrt(v)
    u = np.asarray(u, dtype=np.complex128)
    nb = u.shape[1]
    mb = ((m.reshape(nv * nc, n) * sv[None, :]) @ u).reshape(nv, nc, nb)
    chib = chi0(mb, ev, ec, omega, prefactor)
    out = []
    for cb in chib:
        et = np.eye(n) + u @ (np.linalg.inv(np.eye(nb) - cb) - np.eye(nb)) @ u.conj().T
        out.append(sv[:, None] * et / sv[None, :])
    return np.stack(out)


def screened_w(epsinv_all, vcoul):
    """W_GG'(q) = eps^-1_GG'(q) v(q+G')  (Sec. II)."""
    e = np.asarray(epsinv_all, dtype=np.complex128)
    return e * np.asarray(vcoul, dtype=np.float64)[None, None, :]


def sigma_sx_static(mtxel, epsinv, vcoul, prefactor=1.0):
    """Screened exchange <n|Sigma^SX|n> with the static eps^-1 (Sec. II, the SX
    term of the self-energy with its frequency argument taken at 0):
      -prefactor sum_{n''}^{occ} sum_{G,G'} conj(M_{n''n}(G)) M_{n''n}(G') eps^-1_GG' v(q+G'),
    mtxel [nocc][nband][neps] holding M_{n''n} at -q-G by sphere index G
    (the caller's ordering), epsinv [neps][neps] at omega = 0, vcoul [neps].
    Returns complex [nband].
    """
    m = np.asarray(mtxel, dtype=np.complex128)
    w = np.asarray(epsinv, dtype=np.complex128) * np.asarray(vcoul, dtype=np.float64)[None, :]
    return -prefactor * np.einsum("ang,gh,anh->n", np.conj(m), w, m)


# Modes whose |delta - eps^-1| is at most this are left out of the plasmon-pole
# model (their pole weight is set to zero), as are modes with Re(wtilde^2) <= 0.
GPP_DROP_TOL = 1e-10


def gpp_modes(epsinv, geps, cell, qred, rho_box):
    """Hybertsen-Louie generalized plasmon-pole parameters of the static eps^-1.

    The paper evaluates Sigma with this model (Sec. II, after the COH term, and
    the computational details), which needs only the static eps^-1 and the
    valence density; its parameters are those of the cited Hybertsen-Louie
    model:
      Omega^2_GG' = omega_p^2 (q+G).(q+G') / |q+G|^2 rho(G-G') / rho(0),
      omega_p^2 = 4 pi rho(0),
      wtilde^2_GG' = Omega^2_GG' / (delta_GG' - eps^-1_GG'(q; 0)),
    so that eps^-1(omega) = delta + Omega^2 / (omega^2 - wtilde^2) reproduces the
    static eps^-1 and satisfies the f-sum rule.  wtilde is the principal square
    root.  Modes with |delta - eps^-1| <= GPP_DROP_TOL or Re(wtilde^2) <= 0 are
    dropped (Omega^2 = 0, wtilde = 1).
    rho_box: rho(G) on the FFT box at g mod n.  Returns (omega2, wtilde, keep).
    """
    e = np.asarray(epsinv, dtype=np.complex128)
    g = np.asarray(geps, dtype=np.int64)
    n = e.shape[0]
    qg = 2.0 * np.pi * (g + np.asarray(qred, dtype=np.float64)[None, :]) / np.asarray(cell)
    rho = np.asarray(rho_box, dtype=np.complex128)
    box = np.asarray(rho.shape)
    rho0 = rho[0, 0, 0].real
    wp2 = 4.0 * np.pi * rho0
    # every (G, G') at once: rho at (G - G') mod box, the dot products, the division
    d = np.mod(g[:, None, :] - g[None, :, :], box)
    rho_d = rho[d[..., 0], d[..., 1], d[..., 2]]
    o2 = wp2 * (qg @ qg.T) / (qg * qg).sum(1)[:, None] * rho_d / rho0
    den = np.eye(n) - e
    big = np.abs(den) > GPP_DROP_TOL
    wt2 = np.where(big, o2 / np.where(big, den, 1.0), 0.0)
    keep = big & (wt2.real > 0.0)
    omega2 = np.where(keep, o2, 0.0)
    wtilde = np.where(keep, np.sqrt(np.where(keep, wt2, 1.0)), 1.0 + 0j)
    return omega2, wtilde, keep


def epsinv_gpp(omega2, wtilde, w):
    """The plasmon-pole eps^-1(w) = delta + Omega^2 / (w^2 - wtilde^2) at real w."""
    n = omega2.shape[0]
    return np.eye(n, dtype=np.complex128) + omega2 / (w * w - wtilde * wtilde)


def sigma_gpp(mtxel, en, nocc, vcoul, omega2, wtilde, energies, prefactor=1.0):
    """Diagonal SX and COH matrix elements with the plasmon-pole eps^-1 for one q.

    SX (Sec. II, Eq. sigma_sx), n'' over the first nocc (occupied) states:
      -prefactor sum_{n''} m^H [eps^-1_GPP(E - E_n'') v] m,   m = M_{n''n}.
    COH (Sec. II, Eq. sigma_coh), n'' over every state: with the pole's spectral
    weight -(1/pi) Im eps^-1(w') = Omega^2/(2 wtilde) delta(w' - wtilde) for w' > 0,
      prefactor sum_{n''} m^H [Omega^2 / (2 wtilde (E - E_n'' - wtilde)) v] m
    (reading: the integral runs over w' > 0 and carries v(q+G') as the SX term
    does, as in the Hybertsen-Louie form the paper cites).
    mtxel [nn][nband][neps] (n'' by band n by G), en [nn], energies [nband][ne].
    Each term is built as its full G x G' matrix and contracted: no reordering.
    Returns (sx, coh), each complex [nband][ne].
    """
    m = np.asarray(mtxel, dtype=np.complex128)
    en = np.asarray(en, dtype=np.float64)
    v = np.asarray(vcoul, dtype=np.float64)
    E = np.asarray(energies, dtype=np.float64)
    nn, nband, _ = m.shape
    ne = E.shape[1]
    sx = np.zeros((nband, ne), dtype=np.complex128)
    coh = np.zeros((nband, ne), dtype=np.complex128)
    for b in range(nband):
        for k in range(ne):
            for a in range(nn):
                d = E[b, k] - en[a]
                x = m[a, b]
                c = omega2 / (2.0 * wtilde * (d - wtilde)) * v[None, :]
                coh[b, k] += np.conj(x) @ c @ x
                if a < nocc:
                    f = epsinv_gpp(omega2, wtilde, d) * v[None, :]
                    sx[b, k] -= np.conj(x) @ f @ x
    return prefactor * sx, prefactor * coh


def bse_kernel(mvc, mcc, mvv, vx, w):
    """Exchange and direct kernels of the Bethe-Salpeter equation in the
    Tamm-Dancoff form for one k-point (Sec. II, the K^X and K^D integrals, whose
    spin dependence is the spin trace inside M_nn'):
      K^X_{vc,v'c'} =  sum_G     conj(M_vc(G)) v_x(G) M_v'c'(G),
      K^D_{vc,v'c'} = -sum_{G,G'} conj(M_cc'(G)) W_GG' M_vv'(G').
    Reading: the factors -i and i of the printed integrals are those of the
    Green's-function form; in the eigenvalue problem the exchange enters
    repulsive and the screened direct term attractive, as here.  v_x is the bare
    Coulomb potential with its long-range G = 0 term set to 0 by the caller.
    mvc [nv][nc][N], mcc [nc][nc][N], mvv [nv][nv][N], W [N][N].
    Returns (kx, kd), each [nv*nc][nv*nc] with pair index v*nc + c.
    """
    mvc = np.asarray(mvc, dtype=np.complex128)
    nv, nc, n = mvc.shape
    flat = mvc.reshape(nv * nc, n)
    kx = (np.conj(flat) * np.asarray(vx, dtype=np.float64)[None, :]) @ flat.T
    kd = -np.einsum("cdg,gh,vuh->vcud", np.conj(np.asarray(mcc, dtype=np.complex128)),
                    np.asarray(w, dtype=np.complex128), np.asarray(mvv, dtype=np.complex128))
    return kx, kd.reshape(nv * nc, nv * nc)


def head_overlap(cv, gv, cc, gc):
    """M_vc(G=0) = sum_alpha sum_G conj(c_v^alpha(G)) c_c^alpha(G): the overlap of
    the periodic parts, the G = 0 term of the M_nn' definition (Sec. II).
    Returns [nv][nc] complex128.
    """
    return mtxel_convolution(cv, gv, cc, gc, np.zeros((1, 3), dtype=np.int32))[:, :, 0]


def head_dipole(cv, cc, g, cell, kred, qcart, ev, ec):
    """M_vc(q -> 0, G = 0) from momentum matrix elements at one k-point.

    Sec. II, optical absorption: with the momentum operator standing in for the
    velocity, <v|v|c> = -i (E_c - E_v) <v|r|c>, so to first order in q
    M_vc(q, G=0) = i q.<v|r|c> = q.P_vc / (E_v - E_c), where
    P_vc = sum_alpha sum_G conj(c_v^alpha(G)) (k+G) c_c^alpha(G) and
    k+G = (g + kred) * 2 pi / a (Cartesian, bohr^-1; orthorhombic cell a).
    Valence and conduction coefficients on the same G list g at k.
    Returns [nv][nc] complex128.
    """
    cv = np.asarray(cv, dtype=np.complex128)
    cc = np.asarray(cc, dtype=np.complex128)
    kg = (np.asarray(g, dtype=np.float64) + np.asarray(kred, dtype=np.float64)) * (
        2.0 * np.pi / np.asarray(cell, dtype=np.float64))
    qdot = kg @ np.asarray(qcart, dtype=np.float64)
    p = np.einsum("vsg,g,csg->vc", np.conj(cv), qdot, cc)
    d = np.asarray(ev, dtype=np.float64)[:, None] - np.asarray(ec, dtype=np.float64)[None, :]
    return p / d


def chi0_from_system(sysd, prefactor=1.0, nc=None, method="fft"):
    """Convenience: M then chi0 for a generated system dict."""
    cc = sysd["cc"] if nc is None else sysd["cc"][:nc]
    ec = sysd["ec"] if nc is None else sysd["ec"][:nc]
    if method == "fft":
        m = mtxel_fft(sysd["cv"], sysd["gv"], cc, sysd["gc"], sysd["geps"], sysd["box"])
    else:
        m = mtxel_convolution(sysd["cv"], sysd["gv"], cc, sysd["gc"], sysd["geps"])
    return m, chi0(m, sysd["ev"], ec, sysd["omega"], prefactor)


def rel_f(x, ref):
    """Relative Frobenius error ||x - ref||_F / ||ref||_F."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))
