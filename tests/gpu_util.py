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


def mismatch_reach(gpu_hit, rec, p):
    """Targets whose reuse set holds a pixel where the GPU and the oracle hit
    different triangles (only grazing rays may; compare_hits checks that)."""
    bad = (gpu_hit != rec.hit).astype(np.int32)
    H, W = bad.shape
    out = np.zeros_like(bad, dtype=bool)
    if p.estimator == 0:
        return bad.astype(bool)
    if p.pattern == 0:
        r = p.radius
        pad = np.pad(bad, r)
        for dy in range(2 * r + 1):
            for dx in range(2 * r + 1):
                out |= pad[dy:dy + H, dx:dx + W].astype(bool)
        return out
    gw = 4 if p.group_n == 8 else (2 if p.group_n >= 2 else 1)
    gh = 2 if p.group_n >= 4 else 1
    for y in range(0, H, gh):
        for x in range(0, W, gw):
            if bad[y:y + gh, x:x + gw].any():
                out[y:y + gh, x:x + gw] = True
    return out


def compare_values(gpu, res, region=None, tol=TOL, exclude=None):
    """The GPU estimate must lie within tol of one of the oracle's admissible
    values (one per outcome of each FP32/FP64-ambiguous threshold test).
    Targets in `exclude` (reuse sets holding a differing grazing trace) and
    targets the oracle marks not comparable are counted, not compared."""
    nvar, var = res.nvar, res.var
    if exclude is not None:
        nvar = np.where(exclude, 0, nvar)
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
