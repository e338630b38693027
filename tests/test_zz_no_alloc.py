"""The allocation-free reduction entry point (sph_reduce_static, the library's
own device scratch instead of a caller workspace) against sph_reduce on the
same state, through the C ABI: identical results bit for bit, on two calls in
a row, the second on a smaller particle set (the scratch keeps the first
call's partial sums, which the second must overwrite)."""
import ctypes as C

import numpy as np
import pytest

from paper_2512_05516_amd import inputs

pytestmark = pytest.mark.gpu


def _state(sphmi, ps, n_c):
    from paper_2512_05516_amd.pipeline import Pipeline
    pipe = Pipeline(inputs.pack_aos(ps, "f32"), n_c)
    pipe.bin()
    pipe.convert("full")
    pipe.density()
    pipe.force()
    return pipe


def test_reduce_static_equals_reduce():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_05516_amd import sphmi
    L = sphmi.lib()
    big = inputs.clustered_set(60000, 3, f_blob=0.3)
    sets = [(big, int(np.floor(1.0 / (1.825742 * big.h.max())))), (inputs.small_set(4), 4)]
    for ps, n_c in sets:
        pipe = _state(sphmi, ps, n_c)
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        ref = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        got = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        st = L.sph_reduce(C.byref(pipe.soa.struct), C.byref(pipe.soa.prec),
                          C.byref(pipe.cells.struct), C.c_void_p(ref.data_ptr()),
                          C.c_void_p(pipe.red_ws.data_ptr()), pipe.red_ws.numel(), stream)
        assert st == sphmi.SPH_OK, sphmi.last_error()
        st = L.sph_reduce_static(C.byref(pipe.soa.struct), C.byref(pipe.soa.prec),
                                 C.byref(pipe.cells.struct), C.c_void_p(got.data_ptr()), stream)
        assert st == sphmi.SPH_OK, sphmi.last_error()
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(r)), r
        assert r.tobytes() == g.tobytes(), (ps.n, r, g)
        # the counts are the sums of the loops' per-particle counts
        nn = pipe.soa["NNGB"].cpu().numpy()
        nf = pipe.soa["NFORCE"].cpu().numpy()
        assert g[6] == nn.sum() and g[7] == nf.sum()
        del pipe
        torch.cuda.empty_cache()
    # argument errors are reported before anything is enqueued
    assert L.sph_reduce_static(None, None, None, None, None) == sphmi.SPH_E_INVALID
