"""vl_mass_noalloc, the mass entry point that allocates nothing (partial sums
in the library's static per-GPU array): through the C ABI, against vl_mass of
the same context, bitwise, on two calls in a row, the second with a smaller
input; for FP32 and FP64 fields; and its size limit."""
import numpy as np
import pytest

from paper_2110_13368_amd import binding as vb
from paper_2110_13368_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [vb.VL_F32, vb.VL_F64])
def test_mass_noalloc_equals_vl_mass_twice_second_smaller(precision):
    import torch
    rng = np.random.default_rng(W.SEED_BASE + 9101)
    dtype = "f32" if precision == vb.VL_F32 else "f64"
    big = W.make_sim(rng, (61, 47, 33), (20.0, 20.0, 20.0), 4, dtype=dtype, bc="mixed", n_cells=500,
                     cell_layout="gaussian", sigma=150.0)
    small = W.make_sim(rng, (17, 9, 5), (20.0, 20.0, 20.0), 2, dtype=dtype, bc="neumann", n_cells=30,
                       cell_layout="uniform")
    ctx = vb.Context([big, small], precision=precision, device="cuda:0")
    try:
        ctx.step(3)
        ctx.sync()
        stream = ctx.stream.cuda_stream
        for k in (0, 1):  # the second call has fewer, smaller volumes
            s = ctx.sims[k]
            want = ctx.mass(k)
            out = torch.full((s.n_sub + 3,), -7.0, dtype=torch.float64, device="cuda:0")
            base = ctx.field.data_ptr() + ctx.offsets[k] * ctx.field.element_size()
            print(f"vl_mass_noalloc: sim {k} {s.shape} x {s.n_sub}, precision {precision}", flush=True)
            vb.vl_mass_noalloc(base, precision, s.n_vox, s.n_sub, ctx.strides[k], out.data_ptr(), stream)
            ctx.stream.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got[:s.n_sub], want), (k, got, want)
            assert np.all(got[s.n_sub:] == -7.0)  # nothing written past the volumes
            # and against the field itself (FP64 sum in another order)
            f = ctx.get_field(k).astype(np.float64)
            np.testing.assert_allclose(want, f.reshape(s.n_sub, -1).sum(axis=1), rtol=1e-12)
    finally:
        ctx.close()


def test_mass_noalloc_limit():
    import torch
    field = torch.zeros(65 * 64, dtype=torch.float32, device="cuda:0")
    out = torch.zeros(65, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vb.VoxlodError) as e:
        vb.vl_mass_noalloc(field.data_ptr(), vb.VL_F32, 64, 65, 64, out.data_ptr(), 0)
    assert e.value.code == vb.VL_E_SHAPE and "64 volumes" in vb.vl_last_error()
    vb.vl_mass_noalloc(field.data_ptr(), vb.VL_F32, 64, 64, 64, out.data_ptr(), 0)
    torch.cuda.synchronize()
    assert float(out[:64].abs().sum()) == 0.0
