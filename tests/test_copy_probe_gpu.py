"""The copy probe (vl_copy_probe): every access width and cache policy copies
the bytes exactly, including sizes that end inside a thread's last access
group, and leaves the bytes past the end alone."""
import pytest

from paper_2110_13368_amd import binding as vb

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("width", [4, 8, 16])
@pytest.mark.parametrize("nt", [0, 1, 2, 3])
@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 20) + 16 * 37])
def test_copy_probe_copies_exactly(width, nt, nbytes):
    import torch
    n = nbytes // 4
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (n + 64,), dtype=torch.int32, device="cuda")
    dst = torch.full((n + 64,), 7, dtype=torch.int32, device="cuda")
    print(f"copy probe: width {width}, nt {nt}, {nbytes} bytes", flush=True)
    vb.vl_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, width, nt, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n])
    assert bool((dst[n:] == 7).all())


@pytest.mark.parametrize("width", [4, 16])
@pytest.mark.parametrize("nt", [0, 3])
def test_copy_probe_in_place_leaves_the_buffer_unchanged(width, nt):
    import torch
    nbytes = (1 << 20) + 16 * 37
    n = nbytes // 4
    buf = torch.randint(-2 ** 31, 2 ** 31 - 1, (n + 64,), dtype=torch.int32, device="cuda")
    ref = buf.clone()
    print(f"copy probe in place: width {width}, nt {nt}", flush=True)
    vb.vl_copy_probe(buf.data_ptr(), buf.data_ptr(), nbytes, width, nt, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)


@pytest.mark.parametrize("nbytes", [16, (64 << 10) - 16, (1 << 20) + 16 * 37])
def test_copy_probe_tiles_copy_exactly_and_in_place(nbytes):
    import torch
    n = nbytes // 4
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (n + 64,), dtype=torch.int32, device="cuda")
    dst = torch.full((n + 64,), 7, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    print(f"copy probe tiles: {nbytes} bytes", flush=True)
    vb.vl_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, 16, 4, st)
    ref = src.clone()
    vb.vl_copy_probe(src.data_ptr(), src.data_ptr(), nbytes, 16, 4, st)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n])
    assert bool((dst[n:] == 7).all())
    assert torch.equal(src, ref)
