"""svb_fidelity_noalloc (the entry point that allocates nothing: its partial
sums live in a library-owned device array) against svb_fidelity on the same
registers, through the C ABI: two calls in a row, the second on fewer
registers, both to svb_fidelity's results (the same kernels and FP64 tree:
overlaps bit for bit, fidelities to 1e-15 relative)."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_fidelity_matches_svb_fidelity():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0201042_amd as sv
    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    n, B = 11, 300
    a = sv.Batch(n, B, "c128")
    b = sv.Batch(n, B, "c64")
    rng = np.random.default_rng(7)
    pa = ctypes.c_void_p()
    pb = ctypes.c_void_p()
    _lib.check(L.svb_state(a._h, 0, ctypes.byref(pa)), "svb_state")
    _lib.check(L.svb_state(b._h, 0, ctypes.byref(pb)), "svb_state")
    # random register contents through torch views of the batches' memory
    ta = torch.from_numpy((rng.standard_normal((B << n) * 2)).astype(np.float64)).cuda()
    tb = torch.from_numpy((rng.standard_normal((B << n) * 2)).astype(np.float32)).cuda()
    ta[: 2 << n].zero_()  # register 0 of a: all zero (fidelity 0)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    assert hip.hipMemcpy(pa, ctypes.c_void_p(ta.data_ptr()), (B << n) * 16, 3) == 0
    assert hip.hipMemcpy(pb, ctypes.c_void_p(tb.data_ptr()), (B << n) * 8, 3) == 0
    torch.cuda.synchronize()
    fid_ref, ov_ref = a.fidelity(b)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nregs in (B, 37):
        fid = torch.full((nregs,), -1.0, dtype=torch.float64, device="cuda")
        ov = torch.full((2 * nregs,), -1.0, dtype=torch.float64, device="cuda")
        print("[case] svb_fidelity_noalloc n=%d nregs=%d" % (n, nregs), flush=True)
        rc = L.svb_fidelity_noalloc(n, nregs, 16, pa, 8, pb, ctypes.c_void_p(fid.data_ptr()),
                                    ctypes.c_void_p(ov.data_ptr()), stream)
        assert rc == 0, _lib.load().sv_last_error()
        torch.cuda.synchronize()
        got_ov = ov.cpu().numpy().view(np.complex128)
        got_fid = fid.cpu().numpy()
        assert np.array_equal(got_ov, ov_ref[:nregs])
        assert got_fid[0] == 0.0 and fid_ref[0] == 0.0
        assert np.max(np.abs(got_fid - fid_ref[:nregs]) / np.maximum(np.abs(fid_ref[:nregs]), 1e-300)) <= 1e-15
    # sizes beyond the array are refused before any launch
    assert L.svb_fidelity_noalloc(n, 16385, 16, pa, 8, pb, ctypes.c_void_p(fid.data_ptr()), None, stream) == -1
    a.close()
    b.close()
