"""Elements per workgroup (the paper's element batch size) and the forward
tuner: every launch shape gives the same bits as the default one (the
per-lane arithmetic does not depend on it), unsupported combinations are
refused, and a tuned choice is recorded in the tune table and used by the
default call."""
import numpy as np
import pytest
import torch

import meshgen
from gpu_util import mesh_to_device, vec_to_device

pytestmark = pytest.mark.gpu

fei = pytest.importorskip("paper_1103_0066_amd")

CASES = [("laplace_p1", 2), ("laplace_p1", 3), ("elastic_p1", 2), ("elastic_p1", 3),
         ("laplace_p2", 2), ("laplace_p2", 3)]


def _mesh(form, dim, seed):
    m = (meshgen.square_mesh(23, 0.2, seed, np.float32) if dim == 2
         else meshgen.flatten_elements(meshgen.cube_mesh(7, 6, 5, 0.15, seed), 9, seed + 1))
    mu = lam = None
    if form == "elastic_p1":
        mu, lam = meshgen.lame(m.n_elements, seed + 2)
    return m, mu, lam


@pytest.mark.parametrize("form,dim", CASES)
def test_block_sizes_give_the_default_bits(form, dim):
    m, mu, lam = _mesh(form, dim, 600 + dim)
    coords, conn = mesh_to_device(m)
    mu_d, lam_d = vec_to_device(mu), vec_to_device(lam)
    fei.tune_clear()
    ref = fei.integrate(coords, conn, form, mu_d, lam_d, block_elements=256).cpu().numpy()
    for E in (m.n_elements, 1, 63, 129, 1000):
        sub = conn[:E].contiguous()
        for b in (64, 128, 512):
            A = fei.integrate(coords, sub, form, None if mu_d is None else mu_d[:E].contiguous(),
                              None if lam_d is None else lam_d[:E].contiguous(),
                              block_elements=b).cpu().numpy()
            assert np.array_equal(A.view(np.uint32), ref[:E].view(np.uint32)), (b, E)


def test_block_sizes_refused_where_no_kernel_exists():
    m, mu, lam = _mesh("elastic_p1", 3, 610)
    coords, conn = mesh_to_device(m)
    mu_d, lam_d = vec_to_device(mu), vec_to_device(lam)
    for kw in ({"precision": "fp16x2"}, {"store_rows": 2}):
        with pytest.raises(fei.FeiError) as ex:
            fei.integrate(coords, conn, "elastic_p1", mu_d, lam_d, block_elements=512, **kw)
        assert ex.value.status == fei._lib.FEI_EUNSUPPORTED
    with pytest.raises(fei.FeiError) as ex:
        fei.integrate(coords.double(), conn, "elastic_p1", mu_d, lam_d, block_elements=64)
    assert ex.value.status == fei._lib.FEI_EUNSUPPORTED


def test_tuner_records_and_default_call_uses_it(tmp_path):
    m, mu, lam = _mesh("elastic_p1", 3, 620)
    coords, conn = mesh_to_device(m)
    mu_d, lam_d = vec_to_device(mu), vec_to_device(lam)
    fei.tune_clear()
    try:
        assert fei.tune_lookup("elastic_p1", 3, "fp32", m.n_elements) is None
        r = fei.tune_forward(coords, conn, "elastic_p1", mu_d, lam_d)
        print(f"[tune] {r}", flush=True)
        assert r["candidates"] >= 5 and r["ms"] > 0
        assert fei.tune_lookup("elastic_p1", 3, "fp32", m.n_elements) == r
        A_default = fei.integrate(coords, conn, "elastic_p1", mu_d, lam_d).cpu().numpy()
        A_explicit = fei.integrate(coords, conn, "elastic_p1", mu_d, lam_d,
                                   block_elements=r["block_elements"] or 256,
                                   store_rows=r["store_rows"]).cpu().numpy()
        assert np.array_equal(A_default.view(np.uint32), A_explicit.view(np.uint32))
        # the table persists and reloads
        path = str(tmp_path / "tune.jsonl")
        fei.tune_save(path)
        fei.tune_clear()
        assert fei.tune_lookup("elastic_p1", 3, "fp32", m.n_elements) is None
        fei.tune_load(path)
        assert fei.tune_lookup("elastic_p1", 3, "fp32", m.n_elements)["block_elements"] == \
            r["block_elements"]
        # MFMA precisions tune their staging
        r16 = fei.tune_forward(coords, conn, "elastic_p1", mu_d, lam_d, precision="fp16x2")
        assert r16["candidates"] == 2
    finally:
        fei.tune_clear()
