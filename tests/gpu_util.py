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


def compare_records(gpu_dz, gpu_nz, gpu_hit, rec, o):
    """Where the hits agree: dz = z - o and the oriented normal."""
    same = (gpu_hit == rec.hit) & (rec.hit < oracle.SELF)
    ref_dz = rec.z[same] - o[same].astype(np.float64)
    err = np.linalg.norm(gpu_dz[same].astype(np.float64) - ref_dz, axis=1)
    scale = np.linalg.norm(ref_dz, axis=1)
    # the distance along a ray is ill-conditioned at grazing incidence: allow
    # FP32 error of a few ulps of |dz| divided by |cos| of the hit angle
    cos = np.abs(np.einsum("ij,ij->i", rec.nz[same], ref_dz)) / np.maximum(scale, 1e-30)
    allow = 8e-7 * scale / np.maximum(cos, 1e-3) + 1e-6
    assert (err <= allow).all(), float((err / allow).max())
    nerr = np.abs(gpu_nz[same].astype(np.float64) - rec.nz[same]).max() if same.any() else 0.0
    assert nerr < 1e-5, nerr
    return int(same.sum())


def compare_values(gpu, res, region=None, tol=TOL):
    """The GPU estimate must lie within tol of one of the oracle's admissible
    values (one per outcome of each FP32/FP64-ambiguous threshold test).
    Targets whose reuse set holds a grazing trace are excluded (counted)."""
    if region is not None:
        x0, y0, x1, y1 = region
        gpu = gpu[y0:y1, x0:x1]
        nvar = res.nvar[y0:y1, x0:x1]
        var = res.var[y0:y1, x0:x1]
    else:
        nvar, var = res.nvar, res.var
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
