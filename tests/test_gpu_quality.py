"""The quality harness (quality.py) at a small size: its reference against
the oracle's FP64 quadrature at sampled pixels, and the properties of the
estimators that hold on any scene -- biased reuse lowers the one-sample AO
error, the unbiased estimators converge at the Monte Carlo rate, and
light-sample reuse re-traced over 8 pixels behaves like 8 samples; for
solid-angle shadows and direct illumination, under uniform and bilinear
light sampling, the unbiased estimators converge to the same reference."""
import types

import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ocr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23122_amd as ocr
    ocr.lib()
    return ocr


def _args(**kw):
    a = dict(views=1, ref_spp=256, seeds=2, budget_ao=2.0, budget_shadow=5.0, width=320, height=180,
             light_pdf="uniform")
    a.update(kw)
    return types.SimpleNamespace(**a)


def test_reference_matches_quadrature(ocr):
    import quality
    scene = w.terrain_scene(2)
    bvh = ocr.build_bvh(scene.V, scene.F)
    cam = w.terrain_camera(320, 180)
    view = quality.View(ocr, torch, scene, bvh, cam, "ao", None)
    n = 512
    ref = quality.render(ocr, torch, view, quality.methods("ao")["RT"], 999, n).cpu().numpy()
    sc = oracle.Scene(scene.V, scene.F)
    o, _, kind = oracle.samples(view.gb, oracle.params("ao", "none"))
    rng = np.random.default_rng(4)
    ys, xs = np.nonzero(view.gb.valid)
    pick = rng.choice(len(ys), 12, replace=False)
    for k in pick:
        y, x = int(ys[k]), int(xs[k])
        q = sc.ao_quadrature(o[y, x].astype(np.float64), view.gb.nrm[y, x].astype(np.float64), quality.R_AO,
                             ign=int(view.gb.prim[y, x]), nstrata=192)
        sd = np.sqrt(max(q * (1 - q), 1e-4) / n)
        log(f"    pixel ({x},{y}): reference {ref[y, x]:.4f}, quadrature {q:.4f}")
        assert abs(ref[y, x] - q) < 4.5 * sd + 2e-3


def test_estimator_properties(ocr):
    import quality
    res = quality.evaluate(ocr, torch, "ao", _args())
    log(quality.markdown(res))
    assert res["equal_spp_ratio"]["Occ (8)"] < 0.9
    assert res["equal_spp_ratio"]["Occ (7x7)"] < res["equal_spp_ratio"]["Occ (2)"]
    for n in ("RT", "Occ (8U)", "Occ (7x7U)"):
        c = res["convergence"][n]
        assert c["64"] < 0.08 * c["1"], (n, c)  # ~1/spp, plus the reference's own noise
    sh = quality.evaluate(ocr, torch, "shadow", _args(), 1.0)
    log(quality.markdown(sh))
    assert sh["equal_spp_ratio"]["Light (8U)"] < 0.3
    for n in ("RT", "Occ (8U)"):
        c = sh["convergence"][n]
        assert c["64"] < 0.08 * c["1"], (n, c)


@pytest.mark.parametrize("effect", ["shadow_sa", "di"])
@pytest.mark.parametrize("pdf", ["uniform", "bilinear"])
def test_solid_angle_and_direct_illumination(ocr, effect, pdf):
    import quality
    res = quality.evaluate(ocr, torch, effect, _args(light_pdf=pdf), 4.0)
    log(quality.markdown(res))
    assert "Light (8U)" not in res["ms_per_spp"]
    # unbiased estimators of either sampling density converge to the uniform
    # no-reuse reference at the Monte Carlo rate
    for n in ("RT", "Occ (8U)", "Occ (7x7U)"):
        c = res["convergence"][n]
        assert c["64"] < 0.08 * c["1"], (n, c)
