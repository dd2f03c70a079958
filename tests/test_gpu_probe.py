"""The counter-calibration copies move exactly the bytes they are given, for
every access kind, including sizes that leave a partial workgroup."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_13072_amd import vflb
    vflb.lib()
    return vflb


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 20) + 16 * 37])
def test_copy_probe_copies_every_byte(V, kind, nbytes):
    import torch
    print(f"copy kind {kind}, {nbytes} bytes", flush=True)
    g = torch.Generator(device="cpu").manual_seed(nbytes + kind)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    V.stream_copy(src, dst[:nbytes], st, kind)
    st.synchronize()
    assert torch.equal(dst[:nbytes].cpu(), src.cpu())
    assert int(dst[nbytes:].abs().sum()) == 0
