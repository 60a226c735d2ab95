"""Error bounds shared by the GPU parity tests (test infrastructure)."""
import numpy as np


def _eloc_error_bound(params, N, M, h, smp):
    """FP32 error bound of the product-form local energy, from FP64 values.

    Per flip of site i the ratio is exp(-2 a_i s_i) prod_j n_j with
    n_j = C_ji - s_i t_j S_ji, (C, S) = (cosh 2W, sinh 2W), t = tanh(theta).
    Each factor carries the table rounding, one FMA and one multiply
    (2.5 u (C + |t S|) absolute) and the effect of the FP32 rounding of theta,
    |S| (1 - t^2) N u (|b| + sum |W|); relative to n this grows where C and
    t S nearly cancel (large weights).  The ratios are summed in FP64.
    """
    u = 2.0 ** -24
    a, b = params[:N], params[N:N + M]
    W = params[N + M:].reshape(M, N)
    s = smp.astype(np.float64)
    theta = s @ W.T + b                                  # [n, M]
    t = np.tanh(theta)
    C, S = np.cosh(2 * W), np.sinh(2 * W)                # [M, N]
    dth = N * u * (np.abs(b) + np.abs(W).sum(axis=1))    # [M]
    out = np.zeros(smp.shape[0])
    for i in range(N):
        n = C[:, i][None, :] - s[:, i:i + 1] * t * S[:, i][None, :]
        err = (2.5 * u * (C[:, i][None, :] + np.abs(t * S[:, i][None, :]))
               + np.abs(S[:, i])[None, :] * (1 - t * t) * dth[None, :]) / np.abs(n)
        ratio = np.exp(-2 * a[i] * s[:, i] + np.log(np.abs(n)).sum(axis=1))
        out += abs(h) * ratio * (err.sum(axis=1) + 4 * u)
    return out
