"""dm_match_images_noalloc (the entry point for callers that cannot
allocate device memory) through the C ABI: its matches equal those of
dm_match_images with a caller workspace, bit for bit, on two calls in a row
whose second pair is smaller (the static array keeps the first call's
contents), in FP32 and BF16; pairs whose workspace exceeds the array are
rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1506_07656_amd as dm
import synth

pytestmark = pytest.mark.gpu

NOALLOC_MAX_BYTES = 128 << 20


def call_noalloc(img1: torch.Tensor, img2: torch.Tensor, prm) -> torch.Tensor:
    """The raw C call: caller-owned outputs, no workspace argument."""
    L = dm.lib()
    H1, W1 = img1.shape
    H2, W2 = img2.shape
    cap = dm.plan(W1, H1, W2, H2, prm).max_matches
    buf = torch.full((cap, 5), -7, dtype=torch.int32, device="cuda")
    n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    st = L.dm_match_images_noalloc(ctypes.c_void_p(img1.data_ptr()), W1, H1, img1.stride(0),
                                   ctypes.c_void_p(img2.data_ptr()), W2, H2, img2.stride(0), ctypes.byref(prm),
                                   ctypes.c_void_p(buf.data_ptr()), cap, ctypes.c_void_p(n_out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, (st, L.dm_last_error().decode())
    torch.cuda.synchronize()
    n = int(n_out.item())
    assert 0 < n <= cap
    return buf[:n].clone()


def call_workspace(img1, img2, prm) -> torch.Tensor:
    m = dm.match_images(img1, img2, prm)
    torch.cuda.synchronize()
    return m


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_workspace_entry_point(prec):
    c1 = synth.make_pair("c1")
    big = [torch.from_numpy(np.ascontiguousarray(c1["img1"])).cuda(),
           torch.from_numpy(np.ascontiguousarray(c1["img2"])).cuda()]
    # second call: a smaller pair of other sizes (I 44 x 36, I' 52 x 30)
    small = [torch.from_numpy(np.ascontiguousarray(c1["img1"][10:46, 6:50])).cuda(),
             torch.from_numpy(np.ascontiguousarray(c1["img2"][12:42, 4:56])).cuda()]
    for name, (a, b), mp in (("64x64", big, 32), ("44x36 / 52x30", small, 0)):
        prm = dm.params(precision=prec, max_patch=mp)
        assert dm.plan(a.shape[1], a.shape[0], b.shape[1], b.shape[0], prm).workspace_bytes <= NOALLOC_MAX_BYTES
        got = call_noalloc(a, b, prm).cpu()
        ref = call_workspace(a, b, prm).cpu()
        print(f"{prec} {name}: {len(got)} matches (workspace entry point: {len(ref)})", flush=True)
        assert len(got) == len(ref)
        np.testing.assert_array_equal(got[:, :4].numpy(), ref[:, :4].numpy().astype(np.int32))
        np.testing.assert_array_equal(got[:, 4].view(torch.float32).numpy(), ref[:, 4].numpy().astype(np.float32))


def test_noalloc_rejects_a_pair_beyond_the_array():
    c3 = synth.make_pair("c3")
    a = torch.from_numpy(c3["img1"]).cuda()
    b = torch.from_numpy(c3["img2"]).cuda()
    L = dm.lib()
    prm = dm.params(precision="bf16")
    cap = dm.plan(512, 256, 512, 256, prm).max_matches
    buf = torch.empty((cap, 5), dtype=torch.int32, device="cuda")
    n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    st = L.dm_match_images_noalloc(ctypes.c_void_p(a.data_ptr()), 512, 256, 512, ctypes.c_void_p(b.data_ptr()), 512,
                                   256, 512, ctypes.byref(prm), ctypes.c_void_p(buf.data_ptr()), cap,
                                   ctypes.c_void_p(n_out.data_ptr()), None)
    assert st == -3, st   # DM_ERR_WORKSPACE
    assert "static array" in L.dm_last_error().decode()
    torch.cuda.synchronize()
    assert int(n_out.item()) == -1   # nothing was enqueued
