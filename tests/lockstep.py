"""Lockstep check of the safeguard (Alg. 2: extrapolation and safeguard) along a GPU run.

For every iteration k of a run that recorded its trace and placements, the
oracle takes the GPU's own X^k, forms X^H (the Jacobi step of eq. 5), X~
(eq. 11 with the factor the GPU recorded, or the per-vertex factors) and
f(X~) - f(X^H) (eq. 1, pair by pair), so that the comparison isolates the
GPU's arithmetic of that iteration from the drift of a free run:
  * the GPU's f(X~) - f(X^H) (trace column 2) within 1e-4 of the oracle's
    value or the FP32 band 64 * 2^-24 of its term scale;
  * the GPU's decision (trace column 1) equal to the oracle's outside that band.
The enumerating strategy (Sec. 5.2) checks the kept candidate's difference and
that no candidate beats it by more than the band.
Where the unordered force pass reports bounds U >= f(X~) - f(X^H) >= L
(trace columns 5 and 6) they are compared with the oracle's bounds within 1e-4
or the band of their own term scale, and the decision they took (U <= 0 keeps
X~, L > 0 keeps X^H; column 2 is then NaN) must match the oracle's exact one
outside its band; where the exact difference was summed (after bounds that
left the sign open), column 2 holds it, checked as above.
"""
import numpy as np

import oracle

AMBIG = 64 * 2.0 ** -24


def check_safeguard_lockstep(D, X0, info, omega_vertex=None, enumerate=False, ordering="jacobi"):
    P, T = info["positions"].astype(np.float64), info["trace"]
    checked = 0
    for k in range(len(T)):
        if T[k, 1] == -1.0:  # no extrapolation formed: nothing to decide
            continue
        Xk = np.asarray(X0, dtype=np.float64) if k == 0 else P[k - 1]
        XH = oracle.h_jacobi(D, Xk) if ordering == "jacobi" else oracle.h_exact(D, Xk)
        if enumerate:
            dfs = [oracle.stress_delta(D, XH + c * (XH - Xk), XH) for c in oracle.ENUM_FACTORS[1:]]
            c = T[k, 3]
            df, sc = (0.0, 0.0) if c == 0.0 else dfs[int(round(2 * c)) - 1]
            tol = max(1e-4 * abs(df), AMBIG * sc)
            assert abs(T[k, 2] - df) <= tol, (k, T[k], df, sc)
            best = min([0.0] + [d for d, _ in dfs])
            assert df <= best + max(AMBIG * max(s for _, s in dfs), 1e-4 * abs(best)), (k, df, best)
            checked += 1
            continue
        if omega_vertex is not None:
            XT = XH + (np.asarray(omega_vertex, dtype=np.float64) - 1.0)[:, None] * (XH - Xk)
        else:
            XT = XH + T[k, 3] * (XH - Xk)
        df, sc = oracle.stress_delta(D, XT, XH)
        if T.shape[1] > 6 and np.isfinite(T[k, 5]):
            u, lo, su, q = oracle.stress_delta_bounds(D, XT, XH)
            btol = AMBIG * (su + q)
            assert abs(T[k, 5] - u) <= max(1e-4 * abs(u), btol), (k, T[k, 5], u, su, q)
            if np.isfinite(T[k, 6]):  # (the pass that sums the difference forms U alone)
                assert abs(T[k, 6] - lo) <= max(1e-4 * abs(lo), btol), (k, T[k, 6], lo, su, q)
            if np.isnan(T[k, 2]):  # decided by a bound
                assert (T[k, 5] <= 0.0) if T[k, 1] == 1.0 else (T[k, 6] > 0.0), (k, T[k])
        if not np.isnan(T[k, 2]):
            tol = max(1e-4 * abs(df), AMBIG * sc)
            assert abs(T[k, 2] - df) <= tol, (k, T[k, 2], df, sc)
        if abs(df) > AMBIG * sc:
            assert T[k, 1] == (1.0 if df <= 0.0 else 0.0), (k, T[k, 1], df, sc)
        checked += 1
    return checked
