"""Helpers shared by the GPU parity tests (comparison logic only)."""
import numpy as np

DISCRETE = ("kind", "region", "panel", "gid", "mat", "accept", "process", "trials", "block")


def by_photon(v):
    """Split a vertex array into per-(event, photon) runs, keeping order."""
    key = v["event"].astype(np.int64) * 2 + v["photon"]
    order = np.argsort(key, kind="stable")
    v = v[order]
    key = key[order]
    cut = np.nonzero(np.diff(key))[0] + 1
    return dict(zip(key[np.r_[0, cut]].tolist(), np.split(v, cut)))


def compare_histories(vg, vo, poses, rel=1e-5):
    """Walk RNG-matched histories in lockstep.

    Returns (n_photons, n_diverged, worst_rel_pos, worst_rel_e, failures):
    a photon diverges at its first discrete difference; before that, every
    position must agree to `rel` of its distance from the global origin and
    every energy to `rel` relative.  Panel steps are in the panel frame, so
    their scale is taken from the oracle point mapped back to global."""
    g = by_photon(vg)
    o = by_photon(vo)
    assert set(g) == set(o)
    n_div = 0
    worst_p = worst_e = 0.0
    fails = []
    for k, a in o.items():
        b = g[k]
        n = min(len(a), len(b))
        diverged = len(a) != len(b)
        for i in range(n):
            if any(int(a[f][i]) != int(b[f][i]) for f in DISCRETE):
                diverged = True
                break
            xo = np.array([a["x"][i], a["y"][i], a["z"][i]], np.float64)
            xg = np.array([b["x"][i], b["y"][i], b["z"][i]], np.float64)
            if a["region"][i] == 1 and a["kind"][i] in (0, 2, 4):
                P = poses[a["panel"][i]]
                glob = P[0:3] + xo[0] * P[3:6] + xo[1] * P[6:9] + xo[2] * P[9:12]
                scale = max(np.linalg.norm(glob), 1.0)
            else:
                scale = max(np.linalg.norm(xo), 1.0)
            rp = np.linalg.norm(xo - xg) / scale
            re = abs(a["e"][i] - b["e"][i]) / max(abs(a["e"][i]), 1.0)
            worst_p, worst_e = max(worst_p, rp), max(worst_e, re)
            if rp > rel or re > rel:
                fails.append((k, i, rp, re))
                break
        n_div += diverged
    return len(o), n_div, worst_p, worst_e, fails


def chi2_two_sample(n1, n2, min_count=10):
    """Two-sample chi-square homogeneity over bins (sparse bins pooled)."""
    from scipy import stats
    n1 = np.asarray(n1, np.float64)
    n2 = np.asarray(n2, np.float64)
    N1, N2 = n1.sum(), n2.sum()
    big = (n1 + n2) >= min_count
    a = np.r_[n1[big], n1[~big].sum()]
    b = np.r_[n2[big], n2[~big].sum()]
    keep = (a + b) > 0
    a, b = a[keep], b[keep]
    chi2 = np.sum((np.sqrt(N2 / N1) * a - np.sqrt(N1 / N2) * b) ** 2 / (a + b))
    df = len(a) - 1
    return chi2, df, stats.chi2.sf(chi2, df)
