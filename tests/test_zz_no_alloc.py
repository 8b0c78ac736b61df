"""vx_plot_noalloc (the plot entry point whose workspace is the library's own
device array) against vx_plot with a caller workspace: the same outputs, bit
for bit, on two calls in a row -- a two-pass plan at k = 22 (hash with the
first pass, region passes, group sort, match), then a smaller one-pass plan
at k = 18 -- so the second call runs on the array the first one left
behind.  Also: the size limit and the argument checks."""
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


def _noalloc_buffers(vx, k, threshold=None):
    """Table and output buffers of a k-plot, no workspace."""
    b = vx.alloc_plot(k, threshold)
    nb = b.native()
    nb.workspace = None
    nb.workspace_bytes = 0
    return b, nb


def _same(vx, a, b, what):
    assert torch.equal(a.t1_keys, b.t1_keys), f"{what}: Table-1 keys differ"
    assert torch.equal(a.t1_nonces, b.t1_nonces), f"{what}: Table-1 nonces differ"
    assert torch.equal(a.bucket_offsets, b.bucket_offsets), f"{what}: offsets differ"
    n = vx.t2_count(b)
    assert vx.t2_count(a) == n, f"{what}: |Table 2| differs"
    assert n <= b.t2_capacity
    assert torch.equal(a.t2[:n], b.t2[:n]), f"{what}: Table 2 differs"
    return n


def test_noalloc_equals_vx_plot_on_two_calls(vx):
    from vx_inputs import derive_key
    stream = torch.cuda.current_stream().cuda_stream
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for k, seed in ((22, 7), (18, 8)):
        key = derive_key(seed)
        p = vx.make_params(key, k)
        need = vx.vx_workspace_bytes(p, vx.VX_CALL_PLOT)
        assert 0 < need <= vx.VX_NOALLOC_WORKSPACE_BYTES
        say(f"noalloc: k={k} seed={seed}, workspace {need} bytes, passes {vx.vx_partition_passes(p)}")
        ref = vx.plot(key, k)
        vx.check_plot(ref, what=f"vx_plot k={k}")
        out, nb = _noalloc_buffers(vx, k)
        out.t1_keys.fill_(-1)
        out.t2.fill_(-1)
        status.fill_(-1)
        vx.vx_plot_noalloc(p, nb, None, status.data_ptr(), stream)
        torch.cuda.synchronize()
        assert int(status.item()) == 0, f"k={k}: device status {int(status.item()):#x}"
        n = _same(vx, out, ref, f"k={k}")
        say(f"noalloc: k={k} equal to vx_plot (|T2| = {n})")
    assert vx.vx_partition_passes(vx.make_params(derive_key(7), 22)) >= 2
    assert vx.vx_partition_passes(vx.make_params(derive_key(8), 18)) == 1


def test_noalloc_limits(vx):
    from paper_2606_14007_amd._native import VX_ERR_INVALID_ARG, VX_ERR_WORKSPACE, VxError
    from vx_inputs import derive_key
    stream = torch.cuda.current_stream().cuda_stream
    key = derive_key(9)
    p = vx.make_params(key, 23)
    assert vx.vx_workspace_bytes(p, vx.VX_CALL_PLOT) > vx.VX_NOALLOC_WORKSPACE_BYTES
    out, nb = _noalloc_buffers(vx, 16)
    with pytest.raises(VxError) as e:
        vx.vx_plot_noalloc(p, nb, None, 0, stream)
    assert e.value.status == VX_ERR_WORKSPACE and "vx_plot_noalloc holds" in str(e.value)
    p16 = vx.make_params(key, 16)
    nb.workspace = out.workspace.data_ptr()
    nb.workspace_bytes = out.workspace.numel()
    with pytest.raises(VxError) as e:
        vx.vx_plot_noalloc(p16, nb, None, 0, stream)
    assert e.value.status == VX_ERR_INVALID_ARG
