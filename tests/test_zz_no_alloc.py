"""ce_cluster_edges_noalloc (the entry point whose workspace is the library's static device array) called
through the C ABI gives exactly the outputs of ce_cluster_edges_async with a caller workspace, on two calls
in a row, the second with a smaller input, and refuses an input too large for the static array."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("msf_tail", "msf_head", "msf_w", "sl_left", "sl_right", "sl_w", "sl_size", "pt_cluster", "pt_lambda",
          "cl_id", "cl_parent", "cl_size", "cl_lambda_birth", "cl_stab_hi", "cl_stab_lo", "cl_selected", "labels")


def _noalloc(lib, ce, ins, n, M, V, outs, hdr, time_bits, stream):
    p = ce.make_params(M, V, time_bits=time_bits)
    return lib.ce_cluster_edges_noalloc(*[ctypes.c_void_p(x.data_ptr()) for x in ins], n, ctypes.byref(p),
                                        ctypes.byref(outs.struct), ctypes.c_void_p(hdr.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_equals_the_workspace_call():
    import paper_2311_10337_amd as ce
    lib = ce.load_library()
    lib.ce_cluster_edges_noalloc.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(ce.CeParams),
                                                                     ctypes.POINTER(ce.CeResult), ctypes.c_void_p,
                                                                     ctypes.c_void_p]
    lib.ce_cluster_edges_noalloc.restype = ctypes.c_int
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    M = 5
    for n, V, seed in ((300_000, 15_000, 61), (40_000, 2000, 62)):  # the second call is smaller
        w = synth.plain_tiny(seed=seed, n=n, V=V)
        ins = [torch.from_numpy(a).to(dev) for a in (w.src, w.dst, w.t)]
        a_out, b_out = ce.Outputs(n, M, dev), ce.Outputs(n, M, dev)
        a_hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
        b_hdr = torch.zeros_like(a_hdr)
        for f in FIELDS:
            a_out.t[f].fill_(1)
            b_out.t[f].fill_(1)
        assert _noalloc(lib, ce, ins, n, M, V, a_out, a_hdr, 24, stream) == ce.CE_OK, ce.last_error()
        got = ce.to_numpy(ce.async_result(a_out, n, a_hdr))
        ws = torch.empty(ce.workspace_bytes(n, V, M), dtype=torch.uint8, device=dev)
        ce.cluster_edges_async(*ins, M, V, b_out, ws, b_hdr, time_bits=24)
        ref = ce.to_numpy(ce.async_result(b_out, n, b_hdr))
        assert torch.equal(a_hdr, b_hdr), n
        for f in FIELDS:
            assert np.array_equal(got[f], ref[f]), (n, f)
    # an input whose workspace passes the static array is refused before anything is enqueued
    big = 4_000_000
    ins = [torch.zeros(big, dtype=torch.int32, device=dev), torch.ones(big, dtype=torch.int32, device=dev),
           torch.zeros(big, dtype=torch.int64, device=dev)]
    hdr = torch.zeros(ce.hdr_words(1), dtype=torch.int64, device=dev)
    assert _noalloc(lib, ce, ins, big, M, 2, ce.Outputs(1, M, dev), hdr, 24, stream) == ce.CE_ENOMEM
    assert "static scratch" in ce.last_error()
