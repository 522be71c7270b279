"""The allocation-free reduction (rd_reduce_noalloc) against rd_reduce.

Both run the same kernels in the same order on the same values, so the FP64
mass and energy must agree bit for bit: a grid's field is copied out densely
on the device and reduced without allocation, twice in a row (the second
call on a smaller field, which leaves part of the shared scratch unused),
for every storage type.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1004_0480_amd import rd

pytestmark = pytest.mark.gpu


def dense_device_copy(torch, g, storage):
    """The grid's species 0 as a dense device tensor of its storage type."""
    f32 = torch.empty(g.shape, dtype=torch.float32, device="cuda")
    rd._check(rd.lib().rd_read_field(g.handle, 0, C.c_void_p(f32.data_ptr()), rd.F32, 1))
    # FP32 -> BF16 / FP16 is exact here: the values came from that storage type
    return f32 if storage == "f32" else f32.to(torch.bfloat16 if storage == "bf16" else torch.float16)


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_noalloc_reduction_equals_grid_reduction(storage):
    import torch
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for shape, h in (((37, 45, 130), 0.5), ((5, 3, 70), 2.0)):
        rng = np.random.default_rng(sum(shape))
        field = rng.uniform(-2.0, 3.0, shape)
        g = rd.Grid(shape, 1, h, storage)
        g.set_model(rd_spec(h))
        g.write(0, field)
        want = g.reduce(0)
        dense = dense_device_copy(torch, g, storage)
        g.close()
        rd.reduce_noalloc(dense.data_ptr(), storage, shape, h, out.data_ptr(), stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(storage, shape, want, got)
        assert got[0] == want[0] and got[1] == want[1], (storage, shape, want, got)


def rd_spec(h):
    from paper_1004_0480_amd.workloads import MIRROR, ModelSpec, uniform_bc
    return ModelSpec("diffusion", 1, 0.1 * h * h, h, [[1.0] * 3], uniform_bc(1, MIRROR))


def test_noalloc_reduction_refusals():
    L = rd.lib()
    out = C.c_void_p(16)            # never dereferenced: every call below is refused first
    assert L.rd_reduce_noalloc(None, rd.F32, 4, 4, 4, 1.0, out, None) == rd.EINVAL
    assert L.rd_reduce_noalloc(out, 7, 4, 4, 4, 1.0, out, None) == rd.EINVAL
    assert L.rd_reduce_noalloc(out, rd.F32, 0, 4, 4, 1.0, out, None) == rd.EINVAL
    assert L.rd_reduce_noalloc(out, rd.F32, 1 << 25, 4, 4, 1.0, out, None) == rd.EINVAL
    assert L.rd_reduce_noalloc(out, rd.F32, 1 << 24, 1 << 24, 1 << 24, 1.0, out, None) == rd.EINVAL
    assert L.rd_reduce_noalloc(out, rd.F32, 4, 4, 4, 0.0, out, None) == rd.EINVAL
