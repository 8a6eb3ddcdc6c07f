"""CPU FP64 oracle of the post-BLS statistics of QLP Data Release Notes 003,
Sec. 2.2 items 2-4, and of the complete detection criteria of the paragraph after
that list.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``.  The product path never imports
it, and it shares no code with the HIP kernels.

Definitions followed here, in order (readings where the note is silent are marked):

* trapezoid model (item 2): period P fixed to the detection's; parameters T0
  (mid-transit time), delta (depth), q (duration / P), q_in (ingress duration /
  duration), z (out-of-transit level; the note fits magnitudes, here fluxes, so the
  model is z - delta s).  With dt the time from the nearest mid-transit, D = q P and
  tau = q_in D: s = 1 for |dt| <= D/2 - tau, s = (D/2 - |dt|) / tau on the ingress
  and egress ramps, s = 0 beyond D/2.  Bounds q in [1e-6, 1], q_in in [0, 0.5];
* the fit uses the points (w > 0) within two durations of mid-transit under the
  starting guess (item 2), weighted least squares (weights w), Levenberg-Marquardt
  (reading): start from the BLS mid-time, depth and duration, q_in = 0.2 and z = the
  weighted mean of the fit points outside the starting box; A = J^T W J, g = J^T W r,
  step from (A + lambda diag A) d = g (lambda starts at 1e-3; a parameter whose
  column is zero is held), bounds applied by clamping; a step is kept when chi^2
  falls (lambda / 10), else lambda x 10; stop when a kept step lowers chi^2 by less
  than 1e-10 of it, when lambda exceeds 1e10, or after 60 iterations;
* noise (item 3, reading of the VARTOOLS/Pont et al. estimate): residuals r = y -
  model over every point with w > 0; sigma_w = their standard deviation; bins of
  width D from the first weighted time; sigma_D = standard deviation of the
  non-empty bins' mean residuals, n_bar = points per non-empty bin, sigma_r^2 =
  max(0, sigma_D^2 - sigma_w^2 / n_bar);
* S/N_pink (item 4, Eq. 2) with delta replaced by the trapezoid's depth integral
  over the duration, divided by the duration: delta (1 - q_in) (reading); n_t =
  points with |dt| < D/2, N_t = distinct transit epochs among them; zero residual
  scatter gives S/N_pink = +inf for a positive depth integral (0 without transit);
* candidate: N_t >= 2, S/N_pink > 9 and S/N > 9.
"""
from __future__ import annotations

import math

import numpy as np

Q_MIN, Q_MAX = 1e-6, 1.0
QIN_MAX = 0.5
QIN0 = 0.2
LAMBDA0 = 1e-3
MAX_ITER = 60
REL_TOL = 1e-10
SNR_MIN = 9.0
NPAR = 5          # T0, delta, q, q_in, z


def time_from_mid(t, T0, P):
    """Signed time from the nearest mid-transit: (x - floor(x + 1/2)) P, x = (t - T0)/P."""
    x = (np.asarray(t, np.float64) - T0) / P
    return (x - np.floor(x + 0.5)) * P


def shape(dt, D, tau):
    a = np.abs(dt)
    half = 0.5 * D
    s = np.zeros_like(a)
    s[a <= half - tau] = 1.0
    ramp = (a > half - tau) & (a < half)
    if tau > 0.0:
        s[ramp] = (half - a[ramp]) / tau
    return s


def model(t, P, th):
    T0, delta, q, qin, z = th
    D = q * P
    return z - delta * shape(time_from_mid(t, T0, P), D, qin * D)


def jacobian(t, P, th):
    """d model / d (T0, delta, q, q_in, z); one-sided at the corners (regions by
    the strict inequalities of ``shape``)."""
    T0, delta, q, qin, z = th
    D = q * P
    tau = qin * D
    dt = time_from_mid(t, T0, P)
    a = np.abs(dt)
    half = 0.5 * D
    s = shape(dt, D, tau)
    J = np.zeros((len(dt), NPAR))
    J[:, 1] = -s
    J[:, 4] = 1.0
    ramp = (a > half - tau) & (a < half)
    if tau > 0.0:
        sg = np.sign(dt[ramp])
        ds_da = -1.0 / tau
        # s = (D/2 - a) / tau with tau = q_in D
        ds_dD = 0.5 / tau - (half - a[ramp]) * qin / (tau * tau)
        ds_dqin = -(half - a[ramp]) * D / (tau * tau)
        J[ramp, 0] = -delta * ds_da * (-sg)          # da/dT0 = -sign(dt)
        J[ramp, 2] = -delta * ds_dD * P              # dD/dq = P
        J[ramp, 3] = -delta * ds_dqin
    return J


def _solve(A, g):
    """Cholesky solve of a symmetric positive definite system; None if not SPD."""
    n = len(g)
    L = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            v = A[i, j] - sum(L[i, k] * L[j, k] for k in range(j))
            if i == j:
                if not v > 0.0:
                    return None
                L[i, i] = math.sqrt(v)
            else:
                L[i, j] = v / L[j, j]
    yv = np.zeros(n)
    for i in range(n):
        yv[i] = (g[i] - sum(L[i, k] * yv[k] for k in range(i))) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (yv[i] - sum(L[k, i] * x[k] for k in range(i + 1, n))) / L[i, i]
    return x


def _clamp(th):
    th = np.array(th, np.float64)
    th[2] = min(max(th[2], Q_MIN), Q_MAX)
    th[3] = min(max(th[3], 0.0), QIN_MAX)
    return th


def fit(t, y, w, P, T0, depth, q):
    """Levenberg-Marquardt trapezoid fit; returns (theta, chi2, iterations, n_fit)."""
    t, y, w = (np.asarray(a, np.float64) for a in (t, y, w))
    D0 = q * P
    sel = (w > 0) & (np.abs(time_from_mid(t, T0, P)) <= 2.0 * D0)
    tf, yf, wf = t[sel], y[sel], w[sel]
    if len(tf) == 0:
        return np.array([T0, depth, q, QIN0, np.nan]), np.nan, 0, 0
    out0 = np.abs(time_from_mid(tf, T0, P)) >= 0.5 * D0
    if np.any(out0):
        z0 = float(np.sum(wf[out0] * yf[out0]) / np.sum(wf[out0]))
    else:
        z0 = float(np.sum(wf * yf) / np.sum(wf))
    th = _clamp([T0, depth, q, QIN0, z0])
    r = yf - model(tf, P, th)
    chi2 = float(np.sum(wf * r * r))
    lam = LAMBDA0
    it = 0
    while it < MAX_ITER:
        it += 1
        J = jacobian(tf, P, th)
        A = J.T @ (wf[:, None] * J)
        g = J.T @ (wf * r)
        Ad = A.copy()
        gd = g.copy()
        for i in range(NPAR):
            if A[i, i] == 0.0:          # a parameter the data do not constrain is held
                Ad[i, :] = 0.0
                Ad[:, i] = 0.0
                Ad[i, i] = 1.0
                gd[i] = 0.0
            else:
                Ad[i, i] = A[i, i] * (1.0 + lam)
        d = _solve(Ad, gd)
        if d is None:
            lam *= 10.0
            if lam > 1e10:
                break
            continue
        th2 = _clamp(th + d)
        r2 = yf - model(tf, P, th2)
        chi2b = float(np.sum(wf * r2 * r2))
        if chi2b < chi2:
            done = (chi2 - chi2b) <= REL_TOL * chi2
            th, r, chi2 = th2, r2, chi2b
            lam = max(lam / 10.0, 1e-12)
            if done:
                break
        else:
            lam *= 10.0
            if lam > 1e10:
                break
    return th, chi2, it, int(len(tf))


def noise(t, r, D):
    """(sigma_w, sigma_r) of residuals r on the time scale D."""
    t, r = np.asarray(t, np.float64), np.asarray(r, np.float64)
    n = len(r)
    if n < 2:
        return 0.0, 0.0
    sw = float(np.sqrt(np.sum((r - r.mean()) ** 2) / (n - 1)))
    k = np.floor((t - t[0]) / D).astype(np.int64)
    keys, inv, cnt = np.unique(k, return_inverse=True, return_counts=True)
    means = np.bincount(inv, weights=r) / cnt
    nb = len(keys)
    if nb < 2:
        return sw, 0.0
    sD2 = float(np.sum((means - means.mean()) ** 2) / (nb - 1))
    nbar = n / nb
    return sw, float(math.sqrt(max(0.0, sD2 - sw * sw / nbar)))


def detect(t, y, w, P, T0, depth, q, snr):
    """The fit, noise, S/N_pink and criteria of one star's detection."""
    t, y, w = (np.asarray(a, np.float64) for a in (t, y, w))
    th, chi2, it, nfit = fit(t, y, w, P, T0, depth, q)
    good = w > 0
    tg, yg = t[good], y[good]
    T0f, delta, qf, qin, z = th
    D = qf * P
    r = yg - model(tg, P, th)
    sw, sr = noise(tg, r, D)
    dt = time_from_mid(tg, T0f, P)
    intr = np.abs(dt) < 0.5 * D
    n_t = int(intr.sum())
    N_t = int(len(np.unique(np.floor((tg[intr] - T0f) / P + 0.5)))) if n_t else 0
    dprime = delta * (1.0 - qin)
    den = math.sqrt(sw * sw / n_t + sr * sr / N_t) if n_t and N_t else 0.0
    if den > 0.0:
        snr_pink = dprime / den
    else:                           # no residual scatter (or no transit)
        snr_pink = math.inf if (n_t and dprime > 0.0) else 0.0
    cand = N_t >= 2 and snr_pink > SNR_MIN and snr > SNR_MIN
    return dict(T0=T0f, depth=delta, q=qf, q_in=qin, z=z, chi2=chi2, iterations=it, n_fit=nfit,
                sigma_w=sw, sigma_r=sr, n_t=n_t, N_t=N_t, depth_eff=dprime, snr_pink=snr_pink,
                candidate=bool(cand))
