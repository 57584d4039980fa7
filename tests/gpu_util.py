"""Helpers for the GPU parity tests: run the library through its C-ABI
binding and compare with the oracle under the stated tolerances."""
import math

import numpy as np

import oracle

TOL = 1e-4  # per-pixel absolute tolerance on estimates when the hits agree


def log(msg):
    print(msg, flush=True)


def compare_hits(gpu_hit, rec, valid):
    """Every hit-id mismatch must be a ray the oracle flags as grazing, and
    the mismatches may be at most 1e-5 of the traced rays."""
    traced = valid & (rec.hit != oracle.SELF)
    mism = traced & (gpu_hit != rec.hit)
    unflagged = mism & ~rec.graze.astype(bool)
    n = int(traced.sum())
    stats = dict(rays=n, mismatches=int(mism.sum()), unflagged=int(unflagged.sum()),
                 grazing=int((traced & rec.graze.astype(bool)).sum()))
    assert stats["unflagged"] == 0, stats
    assert stats["mismatches"] <= math.ceil(1e-5 * n), stats
    # self-blocked decisions are FP32-specified on both sides: exact
    assert np.array_equal(gpu_hit[valid] == oracle.SELF, rec.hit[valid] == oracle.SELF)
    return stats


def compare_records(gpu_dz, gpu_nz, gpu_hit, rec, o, scene):
    """Where the hits agree: dz = z - o and the oriented normal."""
    same = (gpu_hit == rec.hit) & (rec.hit < oracle.SELF)
    ref_dz = rec.z[same] - o[same].astype(np.float64)
    err = np.linalg.norm(gpu_dz[same].astype(np.float64) - ref_dz, axis=1)
    scale = np.linalg.norm(ref_dz, axis=1)
    # FP32 error of the watertight test is a few ulps of the vertex distances
    # L = max_v |v - o|, divided by |cos| of the hit angle along the ray
    tri = scene.V.astype(np.float64)[scene.F[rec.hit[same]]]
    L = np.linalg.norm(tri - o[same].astype(np.float64)[:, None, :], axis=2).max(axis=1)
    cos = np.abs(np.einsum("ij,ij->i", rec.nz[same], ref_dz)) / np.maximum(scale, 1e-30)
    allow = 1e-6 * L / np.maximum(cos, 1e-3) + 1e-7
    assert (err <= allow).all(), float((err / allow).max())
    nerr = np.abs(gpu_nz[same].astype(np.float64) - rec.nz[same]).max() if same.any() else 0.0
    assert nerr < 1e-5, nerr
    return int(same.sum())


class ReachMask(np.ndarray):
    """Targets excluded by differing traces, carrying how many targets one
    differing trace can reach (its reuse sets: (2r+1)^2 for a window of
    radius r, N for groups of N, 1 without reuse)."""
    per_trace = 1


def mismatch_reach(gpu_hit, rec, p):
    """Targets whose reuse set holds a pixel where the GPU and the oracle hit
    different triangles (only grazing rays may; compare_hits checks that)."""
    bad = (gpu_hit != rec.hit).astype(np.int32)
    H, W = bad.shape
    out = np.zeros_like(bad, dtype=bool)
    if p.estimator == 0:
        out = bad.astype(bool)
        reach = 1
    elif p.pattern == 0:
        r = p.radius
        pad = np.pad(bad, r)
        for dy in range(2 * r + 1):
            for dx in range(2 * r + 1):
                out |= pad[dy:dy + H, dx:dx + W].astype(bool)
        reach = (2 * r + 1) ** 2
    else:
        gw = 4 if p.group_n == 8 else (2 if p.group_n >= 2 else 1)
        gh = 2 if p.group_n >= 4 else 1
        for y in range(0, H, gh):
            for x in range(0, W, gw):
                if bad[y:y + gh, x:x + gw].any():
                    out[y:y + gh, x:x + gw] = True
        reach = gw * gh
    m = out.view(ReachMask)
    m.per_trace = reach
    return m


# Default budget of targets that may go uncompared (reuse sets holding a
# grazing trace the two sides resolve differently, or more ambiguous pairs
# than the oracle enumerates): 1e-3 of the targets, at least 2, plus the
# reach of the differing traces compare_hits allows (at most 1e-5 of the
# rays, at least one: a differing trace excludes every target whose reuse
# set holds it).  A larger budget is passed explicitly by the few cases
# built to graze (their reason is given where they call this).
MAX_EXCLUDED = 1e-3


def _budget(targets, max_excluded, exclude):
    per = getattr(exclude, "per_trace", 0) if exclude is not None else 0
    return max(2, math.floor(max_excluded * targets)) + per * math.ceil(1e-5 * targets)


def compare_values(gpu, res, region=None, tol=TOL, exclude=None, max_excluded=MAX_EXCLUDED):
    """The GPU estimate must lie within tol of one of the oracle's admissible
    values (one per outcome of each FP32/FP64-ambiguous threshold test).
    Targets in `exclude` (reuse sets holding a differing grazing trace) and
    targets the oracle marks not comparable are counted, not compared; there
    may be at most max_excluded of the targets (and at least 2) of those."""
    nvar, var = res.nvar, res.var
    budget = None
    if exclude is not None:
        budget_of = lambda n: _budget(n, max_excluded, exclude)  # noqa: E731
        nvar = np.where(exclude, 0, nvar)
    else:
        budget_of = lambda n: _budget(n, max_excluded, None)  # noqa: E731
    if region is not None:
        x0, y0, x1, y1 = region
        gpu = gpu[y0:y1, x0:x1]
        nvar = nvar[y0:y1, x0:x1]
        var = var[y0:y1, x0:x1]
    err = np.abs(gpu.astype(np.float64)[..., None] - var)
    err = np.where(np.arange(8)[None, None, :] < nvar[..., None], err, np.inf).min(axis=-1)
    ok = nvar > 0
    stats = dict(targets=int(nvar.size), compared=int(ok.sum()), excluded=int((~ok).sum()),
                 ambiguous=int((nvar > 1).sum()), max_err=float(err[ok].max()) if ok.any() else 0.0,
                 mean_err=float(err[ok].mean()) if ok.any() else 0.0, bad=int((ok & (err > tol)).sum()))
    assert stats["bad"] == 0, stats
    budget = budget_of(stats["targets"])
    assert stats["excluded"] <= budget, (stats, budget)
    return stats


def compare_mean(gpu_mean, results, excludes, tol=TOL, max_excluded=MAX_EXCLUDED):
    """Multi-sample accumulation: gpu_mean must lie within tol of a mean of
    admissible per-sample oracle values, one value per sample (each sample's
    estimate is within tol of one of its admissible values, so their mean is
    within tol of the mean of those values).  Targets excluded or not
    comparable in any sample are counted, not compared."""
    M = len(results)
    nv = np.stack([np.where(ex, 0, r.nvar) for r, ex in zip(results, excludes)])  # [M, H, W]
    var = np.stack([r.var for r in results])  # [M, H, W, 8]
    ok = (nv > 0).all(axis=0)
    single = ok & (nv == 1).all(axis=0)
    g = gpu_mean.astype(np.float64)
    err = np.full(g.shape, np.inf)
    err[single] = np.abs(g[single] - var[:, single, 0].sum(axis=0) / M)
    amb = np.argwhere(ok & ~single)
    for y, x in amb:
        sums = np.zeros(1)
        for s in range(M):
            vals = var[s, y, x, :nv[s, y, x]]
            sums = (sums[:, None] + vals[None, :]).ravel()
        err[y, x] = np.abs(g[y, x] - sums / M).min()
    stats = dict(targets=int(ok.size), compared=int(ok.sum()), excluded=int((~ok).sum()),
                 ambiguous=int(len(amb)), max_err=float(err[ok].max()) if ok.any() else 0.0,
                 bad=int((ok & (err > tol)).sum()))
    assert stats["bad"] == 0, stats
    budget = max(2, math.floor(max_excluded * stats["targets"])) + sum(
        getattr(ex, "per_trace", 0) for ex in excludes) * math.ceil(1e-5 * stats["targets"])
    assert stats["excluded"] <= budget, (stats, budget)
    return stats


def to_np(t):
    return t.detach().cpu().numpy()


def tiles(W, H, n, size, seed=0, margin=8):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x = int(rng.integers(margin, W - size - margin))
        y = int(rng.integers(margin, H - size - margin))
        out.append((x, y, x + size, y + size))
    return out
