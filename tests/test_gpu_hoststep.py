"""Whole time steps with the records in host memory (the pipeline
comparison): the streaming arrangement (host cell list, per-kernel host
gather of the narrowed inputs, host scatter of the outputs), the in-place
arrangement (records to the device once, GPU convert, records back) and the
plain-AoS baseline run the same kernels, so their records must agree bit for
bit; the step's density and force outputs are checked against the oracle."""
import numpy as np
import pytest

from paper_2512_05516_amd import inputs

from helpers import assert_counts, max_rel, oracle_step, rel_rmse

pytestmark = pytest.mark.gpu

DT = 1e-4
FIELDS = ("x", "v", "u", "rho", "wcount", "rho_dh", "f", "P", "c", "nngb", "a", "du", "vsig",
          "nforce")


@pytest.fixture(scope="module")
def sph():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_05516_amd import sphmi
    sphmi.lib()
    return sphmi


def _step(rec, n_c, kind, steps=1, **kw):
    from paper_2512_05516_amd.hoststep import HostStep, pinned_records
    t, view = pinned_records(rec)
    hs = HostStep(t, rec.dtype, n_c, **kw)
    for _ in range(steps):
        hs.step(kind, DT, DT)
    import torch
    torch.cuda.synchronize()
    return view.copy(), hs


def _same(a, b, tag):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (tag, k)


@pytest.mark.parametrize("store", ["fp32", "fp16"])
def test_streaming_equals_inplace(sph, orc, store):
    """Clustered set (uneven cells, ragged chunks), two steps: streaming ==
    in-place bit for bit (the host quantisation is the device's); with FP32
    storage the first step's density and force match the oracle."""
    ps = inputs.clustered_set(20000, 7)
    n_c = int(np.floor(1.0 / (orc.GAMMA_K * ps.h.max())))
    rec = inputs.pack_aos(ps, "f32")
    prec = (sph.precision() if store == "fp32" else
            sph.precision("f16", "bf16", "f16", scale_m=14, scale_h=5, scale_u=0,
                          anchor=sph.ANCHOR_SUB(2)))
    til = sph.tile(32, 2)
    r_in, _ = _step(rec, n_c, "inplace", prec=prec, til=til, sched="grid")
    r_st, hs = _step(rec, n_c, "streaming", prec=prec, til=til, sched="grid", nthreads=5)
    _same(r_in, r_st, store)
    assert hs.pipe.status() == 0
    if store == "fp32":
        ref = inputs.unpack_aos(rec)
        d, f = oracle_step(orc, ref, n_c)
        assert_counts(orc, r_st["nngb"], r_st["nforce"], d["nngb"], f["nforce"], ref, n_c,
                      tag="streaming")
        assert max_rel(r_st["rho"].astype(np.float64), d["rho"]) < 1e-5
        assert rel_rmse(r_st["a"].astype(np.float64), f["a"]) < 1e-5
        assert rel_rmse(r_st["du"].astype(np.float64), f["du"]) < 1e-5
    r_in2, _ = _step(rec, n_c, "inplace", steps=2, prec=prec, til=til, sched="grid")
    r_st2, _ = _step(rec, n_c, "streaming", steps=2, prec=prec, til=til, sched="grid")
    _same(r_in2, r_st2, store + " step 2")
    assert not np.array_equal(r_st2["x"], r_st["x"])


def test_aos_baseline_equals_inplace(sph, orc):
    """The plain-AoS kernels and the FP32 SoA kernels give the same records
    (per-cell launches, default tile), and both match the oracle: counts
    against FP64 brute force, density and force at the FP32 bar."""
    ps = inputs.small_set(12)
    rec = inputs.pack_aos(ps, "f32")
    r_aos, _ = _step(rec, 4, "aos")
    r_in, _ = _step(rec, 4, "inplace")
    _same(r_aos, r_in, "aos")
    ref = inputs.unpack_aos(rec)
    d, f = oracle_step(orc, ref, 4)
    assert_counts(orc, r_aos["nngb"], r_aos["nforce"], d["nngb"], f["nforce"], ref, 4,
                  min_clear=0.98, tag="aos")
    assert max_rel(r_aos["rho"].astype(np.float64), d["rho"]) < 1e-5
    assert rel_rmse(r_aos["a"].astype(np.float64), f["a"]) < 1e-5
    assert rel_rmse(r_aos["du"].astype(np.float64), f["du"]) < 1e-5


def test_streaming_edge_cases(sph, orc):
    """Empty cells and a single particle in a cell: streaming == in-place."""
    ps = inputs.small_set(13)
    keep = np.nonzero(~((ps.x[:, 0] < 0.5) & (ps.x[:, 1] < 0.5)))[0]   # a quarter of cells empty
    keep = np.concatenate([keep, np.nonzero((ps.x[:, 0] < 0.5) & (ps.x[:, 1] < 0.5))[0][:1]])
    sub = ps.subset(np.sort(keep))
    rec = inputs.pack_aos(sub, "f32")
    r_in, _ = _step(rec, 4, "inplace")
    r_st, _ = _step(rec, 4, "streaming")
    _same(r_in, r_st, "edge")
