"""Jones matrices and chains (paper Section 2.2).

parity pinned: identities checked in tests/test_oracle_pins.py (vec trick,
permutation, conjugate-transpose of a chain, identity for an empty side).
"""
import numpy as np

# eq. permutation: vec(G^H) = P conj(vec(G)), P involutory
PERM = np.array([[1, 0, 0, 0],
                 [0, 0, 1, 0],
                 [0, 1, 0, 0],
                 [0, 0, 0, 1]], dtype=np.float64)
PERM_IDX = np.array([0, 2, 1, 3])


def vec(A):
    """Row-major vectorisation of [...,2,2] -> [...,4] (eq. jones)."""
    A = np.asarray(A)
    return A.reshape(A.shape[:-2] + (4,))


def unvec(v):
    """Inverse row-major vectorisation [...,4] -> [...,2,2]."""
    v = np.asarray(v)
    return v.reshape(v.shape[:-1] + (2, 2))


def dagger(A):
    return np.conj(np.swapaxes(A, -1, -2))


def eye2(S):
    out = np.zeros((S, 2, 2), dtype=np.complex128)
    out[:, 0, 0] = 1.0
    out[:, 1, 1] = 1.0
    return out


def beam_beta(term):
    """4 ln 2 / (fwhm nu_ref)^2 of a pointing term's Gaussian beam."""
    fwhm, nu_ref = term.beam
    return 4.0 * np.log(2.0) / (float(fwhm) * float(nu_ref)) ** 2


def term_jones(term, vis, rows, chans, ants, d):
    """Jones matrix of one chain term for antenna `ants` at samples (rows, chans),
    direction d.  The gain is looked up through the term's time/frequency/direction
    maps.  Diagonal terms use only entries XX and YY; a delay term is
    diag(exp(2 pi i nu tau_X), exp(2 pi i nu tau_Y)) at the channel frequency nu;
    a phase-only term diag(exp(i phi_X), exp(i phi_Y)); an amplitude-only term
    diag(a_X, a_Y) with real a (paper Section 2.4, Scenario 1); a delay and
    offset term diag(exp(i (phi0_X + 2 pi nu tau_X)), exp(i (phi0_Y + 2 pi nu
    tau_Y))); a pointing term (Section 2.4, Scenario 3: one parameter pair per
    antenna, a gain that differs by direction) b I with b the term's Gaussian
    beam at direction d seen from the antenna's pointing offset (dl, dm),
    b = exp(-4 ln 2 ((l_d - dl)^2 + (m_d - dm)^2) (nu / (fwhm nu_ref))^2):
    1/2 at half the full width at nu_ref, the width scaling as 1/nu."""
    t = np.asarray(vis.row_time)[rows]
    gt = np.asarray(term.t_map)[t]
    gf = np.asarray(term.f_map)[chans]
    gd = int(np.asarray(term.d_map)[d])
    S = rows.size
    J = np.zeros((S, 2, 2), dtype=np.complex128)
    if term.kind == "pointing":
        u = np.asarray(term.params, dtype=np.float64)[gt, gf, ants, gd]        # [S][2]
        nu = np.asarray(vis.chan_freq, dtype=np.float64)[chans]
        lm = np.asarray(term.dir_lm, dtype=np.float64)[d]
        b = np.exp(-beam_beta(term) * nu ** 2 * ((lm[0] - u[:, 0]) ** 2 + (lm[1] - u[:, 1]) ** 2))
        J[:, 0, 0] = b
        J[:, 1, 1] = b
    elif term.kind == "delay_offset":
        u = np.asarray(term.params, dtype=np.float64)[gt, gf, ants, gd]        # [S][4]
        nu = np.asarray(vis.chan_freq, dtype=np.float64)[chans]
        J[:, 0, 0] = np.exp(1j * (u[:, 0] + 2.0 * np.pi * nu * u[:, 1]))
        J[:, 1, 1] = np.exp(1j * (u[:, 2] + 2.0 * np.pi * nu * u[:, 3]))
    elif term.kind == "delay":
        tau = np.asarray(term.params, dtype=np.float64)[gt, gf, ants, gd]      # [S][2]
        nu = np.asarray(vis.chan_freq, dtype=np.float64)[chans]
        J[:, 0, 0] = np.exp(2j * np.pi * nu * tau[:, 0])
        J[:, 1, 1] = np.exp(2j * np.pi * nu * tau[:, 1])
    elif term.kind == "phase":
        phi = np.asarray(term.params, dtype=np.float64)[gt, gf, ants, gd]      # [S][2]
        J[:, 0, 0] = np.exp(1j * phi[:, 0])
        J[:, 1, 1] = np.exp(1j * phi[:, 1])
    elif term.kind == "amplitude":
        amp = np.asarray(term.params, dtype=np.float64)[gt, gf, ants, gd]      # [S][2]
        J[:, 0, 0] = amp[:, 0]
        J[:, 1, 1] = amp[:, 1]
    else:
        g = np.asarray(term.gains, dtype=np.complex128)[gt, gf, ants, gd]      # [S][4]
        if term.kind == "diag":
            J[:, 0, 0] = g[:, 0]
            J[:, 1, 1] = g[:, 3]
        else:
            J[:] = unvec(g)
    return J


def chain_product(chain, vis, rows, chans, ants, d, j0, j1):
    """Product G_j0 G_j0+1 ... G_j1-1 (eq. joneschain); the empty product is I
    (eq. jonesfactor)."""
    C = eye2(rows.size)
    for j in range(j0, j1):
        C = C @ term_jones(chain[j], vis, rows, chans, ants, d)
    return C
