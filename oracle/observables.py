"""S-matrix, phase shifts, kinematics and the total cross section (test infrastructure only).

Conventions:
* on-shell S = 1 - i pi p t(p,p) for reduced t (App. A, the S-T relation,
  with the phase-space factor of the <k'|k> = delta/(k'k) normalisation);
  uncoupled S = exp(2 i delta) (App. A);
* the packet T-matrix maps to the continuum as t(q,q) = f(q)^2 T_kk/(N_k q^2)
  (Sec. 3.1, operator transfer between the packet and continuum bases): for
  momentum packets T_kk/(dk_k q^2) at the bin midpoint q = kbar_k (Sec. 3.2,
  choice of on-shell q);
* Stapp parametrisation of the coupled 2x2 S (App. A): S_11 = cos(2 eps)
  exp(2 i delta_-), S_22 = cos(2 eps) exp(2 i delta_+),
  S_12 = S_21 = i sin(2 eps) exp(i (delta_- + delta_+));
* phase shifts are principal values in (-90, 90] degrees (Sec. 5.1), compared
  modulo 180 degrees;
* sigma_tot from the optical theorem in partial waves,
  sigma = (pi/(2 p^2)) sum_(s,l,J) (2J+1) (1 - Re S_ll), every (s,l,J) once
  (App. A, total cross section); 1 fm^2 = 10 mb;
* phase shifts between bin midpoints are linearly interpolated in q
  (Sec. 5.1.1, mid-point interpolation) after unwrapping modulo 180 degrees;
* T_lab -> p non-relativistically with equal masses: p = sqrt(m_N T_lab / 2)/(hbar c).

Pins: Stapp round trip, uncoupled reduction of sigma to (pi/p^2) sin^2 delta,
S-matrix unitarity of the exact solvers, interpolation of linear data.
"""
from __future__ import annotations

import numpy as np

M_N_MEV = 938.918
HBARC_MEV_FM = 197.327


def tlab_to_p(tlab_mev):
    return np.sqrt(M_N_MEV * np.asarray(tlab_mev, dtype=np.float64) / 2.0) / HBARC_MEV_FM


def s_matrix(t_wp: np.ndarray, norm: np.ndarray, q: np.ndarray, f2=None) -> np.ndarray:
    """S(q_k) = 1 - i pi q t,  t = f(q)^2 T/(N_k q^2), for T of shape (N, K, K).

    norm: the packet normalisation N_k (dk_k for momentum packets), q: the
    on-shell momenta, f2: f(q)^2 (None: 1, momentum packets)."""
    n_ch = t_wp.shape[1]
    f2 = np.ones_like(q) if f2 is None else np.asarray(f2, dtype=np.float64)
    t = t_wp * (f2 / (norm * q * q))[:, None, None]
    return np.eye(n_ch)[None, :, :] - 1j * np.pi * q[:, None, None] * t


def s_from_t_continuum(t: np.ndarray, p) -> np.ndarray:
    """S for a continuum on-shell t (K x K or (..., K, K)) at momentum p."""
    t = np.asarray(t)
    n_ch = t.shape[-1]
    return np.eye(n_ch) - 1j * np.pi * np.asarray(p)[..., None, None] * t


def phase_shifts(s: np.ndarray) -> dict:
    """delta (degrees) per channel, Stapp mixing angle eps_J ("mix") for K = 2, and 1 - |S_ll|."""
    n_ch = s.shape[-1]
    delta = np.empty(s.shape[:-2] + (n_ch,))
    for a in range(n_ch):
        delta[..., a] = 0.5 * np.angle(s[..., a, a])
    out = {"s_dev": 1.0 - np.abs(np.stack([s[..., a, a] for a in range(n_ch)], axis=-1))}
    if n_ch == 2:
        s12 = 0.5 * (s[..., 0, 1] + s[..., 1, 0])
        x = np.imag(s12 * np.exp(-1j * (delta[..., 0] + delta[..., 1])))
        out["mix"] = np.degrees(0.5 * np.arcsin(np.clip(x, -1.0, 1.0)))
    else:
        out["mix"] = None
    out["delta"] = np.degrees(delta)
    return out


def stapp_s(delta_m_deg, delta_p_deg, eps_deg) -> np.ndarray:
    """Unitary 2x2 S from Stapp parameters (App. A)."""
    dm, dp, e = (np.radians(np.asarray(x, dtype=np.float64)) for x in (delta_m_deg, delta_p_deg, eps_deg))
    s = np.empty(np.shape(dm) + (2, 2), dtype=np.complex128)
    s[..., 0, 0] = np.cos(2 * e) * np.exp(2j * dm)
    s[..., 1, 1] = np.cos(2 * e) * np.exp(2j * dp)
    s[..., 0, 1] = s[..., 1, 0] = 1j * np.sin(2 * e) * np.exp(1j * (dm + dp))
    return s


def unwrap_deg(delta_deg: np.ndarray):
    """Sequential unwrap modulo 180 degrees from the lowest bin upwards.

    Returns the unwrapped values and the integer number of 180-degree shifts
    applied to each bin.
    """
    d = np.asarray(delta_deg, dtype=np.float64).copy()
    shifts = np.zeros(d.shape, dtype=np.int64)
    for i in range(1, d.shape[0]):
        s = np.round((d[i - 1] - d[i]) / 180.0)
        d[i] += 180.0 * s
        shifts[i] = s.astype(np.int64)
    return d, shifts


def interpolate(kbar: np.ndarray, y: np.ndarray, p, k_max: float):
    """Piecewise-linear y(p) between consecutive midpoints (Sec. 5.1.1).

    Below the first and above the last midpoint the end segments are
    extrapolated; p above the mesh cut-off k_max is an error.
    """
    p = np.atleast_1d(np.asarray(p, dtype=np.float64))
    if np.any(p > k_max) or np.any(p <= 0):
        raise ValueError("on-shell momentum outside (0, k_max]")
    i = np.clip(np.searchsorted(kbar, p, side="right"), 1, kbar.size - 1)
    x0, x1 = kbar[i - 1], kbar[i]
    y0, y1 = y[i - 1], y[i]
    return y0 + (y1 - y0) * (p - x0) / (x1 - x0)


def interpolation_points(k_bounds, frac: float):
    """Abscissae q_i = k_{i-1} + frac (k_i - k_{i-1}) to which the bin values
    are assigned before interpolating (Sec. 5.1.1, the interpolation point
    n/m of a bin; frac = n/m = 1/2 is the midpoint)."""
    k = np.asarray(k_bounds, dtype=np.float64)
    if not (0.0 <= frac <= 1.0):
        raise ValueError("frac must lie in [0, 1]")
    return k[:-1] + frac * np.diff(k)


def sigma_band(channels, tlab_mev, fracs):
    """Lowest and highest total cross section (mb) over interpolation points.

    channels: iterable of (J, delta_deg (N, K), eps_deg (N,) or None,
    k_bounds); for every frac in fracs the bin phases are placed at
    interpolation_points(k_bounds, frac) and sigma_tot is evaluated; returns
    (min, max) over fracs per T_lab (Sec. 5.1.1: the bands of varying the
    interpolation point, m = 10 and n = 0.1, 1, 2, ..., 9, 9.9 there)."""
    chans = [(J, d, e, np.asarray(k, dtype=np.float64)) for J, d, e, k in channels]
    sig = np.stack([sigma_tot([(J, d, e, interpolation_points(k, f), k[-1]) for J, d, e, k in chans], None,
                              tlab_mev, None) for f in fracs])
    return sig.min(axis=0), sig.max(axis=0)


def channel_loss(delta_deg: np.ndarray, eps_deg, kbar: np.ndarray, p, k_max: float):
    """sum_l (1 - Re S_ll) at momenta p from one channel's bin phase shifts.

    delta_deg has shape (N, K).  For K = 2 the mixing angle's sign follows the
    180-degree shifts applied to delta_- and delta_+ during unwrapping, so that
    it stays tied to the unwrapped phases.
    """
    n_ch = delta_deg.shape[1]
    ds, sh = [], []
    for a in range(n_ch):
        d, s = unwrap_deg(delta_deg[:, a])
        ds.append(d)
        sh.append(s)
    total = 0.0
    if n_ch == 1:
        dl = np.radians(interpolate(kbar, ds[0], p, k_max))
        total = 1.0 - np.cos(2.0 * dl)
    else:
        sign = np.where((sh[0] + sh[1]) % 2 == 0, 1.0, -1.0)
        e = np.radians(interpolate(kbar, sign * np.asarray(eps_deg), p, k_max))
        for a in range(2):
            dl = np.radians(interpolate(kbar, ds[a], p, k_max))
            total = total + 1.0 - np.cos(2.0 * e) * np.cos(2.0 * dl)
    return total


def sigma_from_s(channels, p) -> float:
    """Total cross section in mb at momentum p from on-shell S matrices.

    channels: iterable of (J, S) with S the K x K on-shell S-matrix of the
    channel at p (App. A, optical theorem in partial waves, as in sigma_tot
    but with no interpolation: the S matrices are those at p itself).
    """
    acc = 0.0
    for J, s in channels:
        s = np.atleast_2d(np.asarray(s))
        acc += (2 * J + 1) * float(np.sum(1.0 - np.real(np.diag(s))))
    return 10.0 * np.pi / (2.0 * p * p) * acc


def sigma_tot(channels, kbar, tlab_mev, k_max) -> np.ndarray:
    """Total cross section in mb at the given T_lab values.

    channels: iterable of (J, delta_deg (N, K), eps_deg (N,) or None), all on
    the bins with midpoints kbar and top momentum k_max, or of
    (J, delta_deg, eps_deg, kbar_c, k_max_c) for channels on their own bins
    (then kbar and k_max may be None).
    """
    p = tlab_to_p(tlab_mev)
    acc = np.zeros_like(p)
    for ch in channels:
        J, delta_deg, eps_deg = ch[:3]
        kb, km = (ch[3], ch[4]) if len(ch) > 3 else (kbar, k_max)
        acc = acc + (2 * J + 1) * channel_loss(np.asarray(delta_deg), eps_deg, kb, p, km)
    return 10.0 * np.pi / (2.0 * p * p) * acc
