"""WPCD in plain FP64 NumPy, one channel at a time (test infrastructure only).

Conventions (read from Sec. 2 and Sec. 3 of the paper):
* partial-wave states <k'|k> = delta(k'-k)/(k'k); reduced units, energies are
  E = k^2 in fm^-2 and the potential U is in fm (no 2/pi in the LS kernel);
* momentum wave packets, f(k) = 1 and N_i = dk_i, or energy wave packets,
  f(k) = sqrt(k/mu) and N_i = dE_i (Sec. 3.1, definition of the free wave
  packet and the normalisation stated after its eigenvalue equations).  In
  the reduced units used here E = k^2, i.e. hbar^2/(2 mu) = 1, so
  f(k)^2 dk = dE: f(k) = sqrt(2k) and N_i = k_i^2 - k_{i-1}^2;
* coupled channels use K = 2 degenerate copies of the free basis, one per
  orbital l, ordered channel-major: row (a, i) -> a*N + i (Sec. 3.1, coupled
  channels paragraph).

Pins (tests/test_oracle_*.py): projection against closed-form polynomial
integrals and the rank-1 Yamaguchi structure; H0 against <k^2> over a bin; the
resolvent table against numerical double integrals and its far-bin limit; the
SWP boundaries against hand examples; T against V = 0, the Born limit and
N_WP -> infinity convergence to the matrix-inversion solver and the Yamaguchi
closed form.  Finite-N_WP values themselves have no external reference:
at a fixed N_WP the oracle *is* the reference ("parity unpinned" beyond the
pins listed).
"""
from __future__ import annotations

import numpy as np


class WPCDError(ValueError):
    """A channel the method cannot process (degenerate family or energy)."""


# ---------------------------------------------------------------- step 1: bins
def bins(k_bounds):
    """Bin widths dk_i, midpoints kbar_i and boundary energies E_j = k_j^2.

    Bins D_i = [k_{i-1}, k_i] (Sec. 3.1, non-overlapping bins; Sec. 3.2 for the
    midpoint definition).
    """
    k = np.asarray(k_bounds, dtype=np.float64)
    if k.ndim != 1 or k.size < 3 or k[0] != 0.0 or np.any(np.diff(k) <= 0):
        raise WPCDError("k_bounds must start at 0 and increase strictly")
    return np.diff(k), 0.5 * (k[1:] + k[:-1]), k * k


def gauss_nodes(k_bounds, n_gauss: int):
    """Gauss-Legendre nodes/weights mapped into every bin, bin-major."""
    k = np.asarray(k_bounds, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(n_gauss)
    a, b = k[:-1, None], k[1:, None]
    nodes = 0.5 * (b - a) * x[None, :] + 0.5 * (b + a)
    weights = 0.5 * (b - a) * w[None, :]
    return nodes.ravel(), weights.ravel()


PACKETS = ("momentum", "energy")


def _check_packet(packet: str):
    if packet not in PACKETS:
        raise WPCDError(f"packet must be one of {PACKETS}, got {packet!r}")


def h0_diagonal(k_bounds, packet: str = "momentum"):
    """e_i = <x_i|k^2|x_i> = (1/N_i) int_{D_i} k^2 f(k)^2 dk.

    The free Hamiltonian is diagonal in the packet basis because bins do not
    overlap (Sec. 3.1, free wave packets and their free-Hamiltonian
    eigenvalue).  Momentum packets: the bin average of k^2 over k,
    (k_{i-1}^2 + k_{i-1} k_i + k_i^2)/3 (see the reading list for the choice
    of <k^2>); energy packets: the bin average of E over E, i.e. the energy
    midpoint E_{i-1} + dE_i/2 = (k_{i-1}^2 + k_i^2)/2, the eigenvalue the
    paper states for them.
    """
    _check_packet(packet)
    k = np.asarray(k_bounds, dtype=np.float64)
    a, b = k[:-1], k[1:]
    if packet == "energy":
        return 0.5 * (a * a + b * b)
    return (a * a + a * b + b * b) / 3.0


def packet_weight(k, packet: str = "momentum"):
    """f(k) of the free packet definition: 1 (momentum) or sqrt(2k) (energy)."""
    _check_packet(packet)
    k = np.asarray(k, dtype=np.float64)
    return np.ones_like(k) if packet == "momentum" else np.sqrt(2.0 * k)


def packet_norm(k_bounds, packet: str = "momentum"):
    """N_i: dk_i (momentum packets) or dE_i = k_i^2 - k_{i-1}^2 (energy packets)."""
    _check_packet(packet)
    k = np.asarray(k_bounds, dtype=np.float64)
    return np.diff(k) if packet == "momentum" else np.diff(k * k)


def onshell_momenta(k_bounds, packet: str = "momentum"):
    """The on-shell momentum q_k of each bin: the one whose energy is the
    packet's free eigenvalue (Sec. 3.2, choice of q after the five steps):
    the momentum midpoint kbar_k for momentum packets (their momentum
    eigenvalue k_{k-1} + dk_k/2), sqrt(e_k) = sqrt((k_{k-1}^2 + k_k^2)/2) for
    energy packets (their energy eigenvalue E_{k-1} + dE_k/2)."""
    _check_packet(packet)
    if packet == "momentum":
        return bins(k_bounds)[1]
    return np.sqrt(h0_diagonal(k_bounds, "energy"))


# ------------------------------------------------------- step 1b: projection
def projection_matrix(k_bounds, n_gauss: int, n_ch: int, packet: str = "momentum") -> np.ndarray:
    """P with V = P^T U P: P[(a,alpha),(a,i)] = w_alpha k_alpha f(k_alpha) / sqrt(N_i).

    From the double-bin-integral definition of <x_i|v|x_j> (Sec. 3.2,
    wave-packet potential matrix), evaluated with the per-bin Gauss rule.
    With one node per bin (n_gauss = 1: the midpoint kbar_i, weight dk_i) this
    is the paper's midpoint approximation, which for momentum packets reads
    V_ij = kbar_i kbar_j sqrt(dk_i dk_j) U(kbar_i, kbar_j).
    """
    k = np.asarray(k_bounds, dtype=np.float64)
    n = k.size - 1
    nodes, w = gauss_nodes(k, n_gauss)
    norm = packet_norm(k, packet)
    f = packet_weight(nodes, packet)
    m = n * n_gauss
    p = np.zeros((n_ch * m, n_ch * n))
    for a in range(n_ch):
        for i in range(n):
            sl = slice(i * n_gauss, (i + 1) * n_gauss)
            rows = slice(a * m + i * n_gauss, a * m + (i + 1) * n_gauss)
            p[rows, a * n + i] = w[sl] * nodes[sl] * f[sl] / np.sqrt(norm[i])
    return p


def project(k_bounds, n_gauss: int, u_fine: np.ndarray, n_ch: int, packet: str = "momentum") -> np.ndarray:
    """Wave-packet potential matrix V (n_ch*N square) from U at the Gauss nodes."""
    p = projection_matrix(k_bounds, n_gauss, n_ch, packet)
    u = np.asarray(u_fine, dtype=np.float64)
    if u.shape != (p.shape[0], p.shape[0]):
        raise WPCDError(f"u_fine must be {p.shape[0]} square, got {u.shape}")
    return p.T @ u @ p


def hamiltonian(k_bounds, v: np.ndarray, n_ch: int, packet: str = "momentum") -> np.ndarray:
    """H = H0 + V with H0 repeated once per coupled channel (Sec. 3.1)."""
    e = np.tile(h0_diagonal(k_bounds, packet), n_ch)
    return np.diag(e) + v


# ----------------------------------------------------------- step 2: diagonalise
def diagonalise(h: np.ndarray):
    """Ascending eigenvalues and orthonormal eigenvectors, H = C D C^T (Sec. 3.1)."""
    return np.linalg.eigh(h)


# ------------------------------------------------- step 3: SWP bin boundaries
def swp_bins(eps: np.ndarray, n_ch: int, e_top: float = np.inf):
    """Energy bins [lo, hi] of the scattering wave packets.

    Eigenvalues eps < 0 are bound states and eigenvalues above the top of the
    free continuum, eps > e_top = k_N^2, are discrete states of the cut-off
    Hamiltonian; neither gets a bin.  The remaining ones, in ascending order,
    are dealt round-robin into n_ch families (Sec. 3.1, coupled channels: each
    free level splits into n_ch scattering levels, which do not mix across
    levels).  Within a family with eigenvalues e_1 < ... < e_n the boundaries
    are B_1 = 0, B_i = (e_{i-1} + e_i)/2 and B_{n+1} = e_n + (B_n - B_{n-1})/2
    (Sec. 3.1, scheme for the pseudostate bin boundaries).  Returns lo, hi (NaN
    for discrete states) and the discrete-state mask.
    """
    eps = np.asarray(eps, dtype=np.float64)
    if np.any(eps == 0.0):
        raise WPCDError("eigenvalue exactly zero: neither bound nor scattering")
    if np.any(np.diff(eps) < 0):
        raise WPCDError("eigenvalues must be ascending")
    bound = (eps < 0.0) | (eps > e_top)
    pos = np.flatnonzero(~bound)
    lo = np.full(eps.size, np.nan)
    hi = np.full(eps.size, np.nan)
    for kappa in range(n_ch):
        fam = pos[kappa::n_ch]
        e = eps[fam]
        nf = e.size
        if nf < 2:
            raise WPCDError("a scattering family needs at least two members")
        b = np.empty(nf + 1)
        b[0] = 0.0
        b[1:nf] = 0.5 * (e[:-1] + e[1:])
        b[nf] = e[-1] + 0.5 * (b[nf - 1] - b[nf - 2])
        lo[fam] = b[:-1]
        hi[fam] = b[1:]
    if np.any(hi[~bound] <= lo[~bound]):
        raise WPCDError("zero-width scattering bin")
    return lo, hi, bound


# ------------------------------------------------ step 4: averaged resolvent
def _xlogx(x):
    ax = np.abs(x)
    out = np.zeros_like(x)
    nz = ax > 0
    out[nz] = x[nz] * np.log(ax[nz])
    return out


def resolvent_table(k_bounds, eps, lo, hi, bound) -> np.ndarray:
    """gbar[k, m]: <z_m|g(E)|z_m> averaged over E in the free bin k.

    Scattering packet m is an energy packet on [c, d] = [lo_m, hi_m], so
    <z_m|g(E)|z_m> = (1/(d-c)) int_c^d dE'/(E - E' + i0) (App. B); averaging E
    over the free bin [a, b] = [k_{k-1}^2, k_k^2] (Sec. 3.2, energy averaging)
    gives (1/((b-a)(d-c))) [F(b-c) - F(a-c) - F(b-d) + F(a-d)
    - i pi |[a,b] & [c,d]|] with F(x) = x ln|x|, F(0) = 0.  A discrete state
    (bound, or above the free continuum) contributes 1/(E - eps_m) (Sec. 3.2,
    bound-state term of the LS equation in the packet basis), whose bin average
    is ln((b - eps)/(a - eps))/(b - a).
    """
    _, _, e_b = bins(k_bounds)
    a = e_b[:-1, None]
    b = e_b[1:, None]
    de = b - a
    n = eps.size
    g = np.zeros((a.shape[0], n), dtype=np.complex128)
    sc = ~bound
    if np.any(sc):
        c = lo[None, sc]
        d = hi[None, sc]
        re = (_xlogx(b - c) - _xlogx(a - c) - _xlogx(b - d) + _xlogx(a - d)) / (de * (d - c))
        ov = np.clip(np.minimum(b, d) - np.maximum(a, c), 0.0, None)
        g[:, sc] = re - 1j * np.pi * ov / (de * (d - c))
    if np.any(bound):
        eb = eps[None, bound]
        g[:, bound] = np.log((b - eb) / (a - eb)) / de
    return g


# ---------------------------------------------- step 5: T at all bin energies
def tmatrix(v: np.ndarray, c: np.ndarray, gbar: np.ndarray, n_ch: int) -> np.ndarray:
    """On-shell T_ab(k) = V_{(a,k),(b,k)} + sum_m (VC)_{(a,k),m} gbar_km (VC)_{(b,k),m}.

    This is the LS equation with the full resolvent in the packet basis
    (Sec. 3.2, step 5) evaluated on the diagonal bin k for every bin at once.
    Returns T with shape (N, n_ch, n_ch), complex.
    """
    n = gbar.shape[0]
    vc = v @ c
    t = np.empty((n, n_ch, n_ch), dtype=np.complex128)
    kk = np.arange(n)
    for a in range(n_ch):
        for b in range(n_ch):
            ra, rb = a * n + kk, b * n + kk
            t[:, a, b] = v[ra, rb] + np.sum(vc[ra, :] * gbar * vc[rb, :], axis=1)
    return t


def solve_channel(k_bounds, n_gauss: int, u_fine: np.ndarray, n_ch: int, packet: str = "momentum") -> dict:
    """Steps 1-5 of the method plus S-matrix phase shifts for one channel.

    packet selects momentum (default) or energy wave packets; "q" in the
    result holds the on-shell momentum of every bin (onshell_momenta)."""
    from . import observables

    q = onshell_momenta(k_bounds, packet)
    v = project(k_bounds, n_gauss, u_fine, n_ch, packet)
    h = hamiltonian(k_bounds, v, n_ch, packet)
    evals, c = diagonalise(h)
    lo, hi, bound = swp_bins(evals, n_ch, float(np.asarray(k_bounds)[-1]) ** 2)
    g = resolvent_table(k_bounds, evals, lo, hi, bound)
    t = tmatrix(v, c, g, n_ch)
    s = observables.s_matrix(t, packet_norm(k_bounds, packet), q, packet_weight(q, packet) ** 2)
    ph = observables.phase_shifts(s)
    return {"v": v, "h": h, "evals": evals, "evecs": c, "lo": lo, "hi": hi, "bound": bound,
            "gbar": g, "t": t, "s": s, "delta": ph["delta"], "mix": ph["mix"],
            "s_dev": ph["s_dev"], "q": q}
