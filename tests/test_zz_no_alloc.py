"""The convolution entry point that allocates nothing (lar_fftconv_noalloc,
for callers that cannot allocate device memory) against lar_fftconv, through
the C ABI: the same kernels on the same inputs give bit-identical waveforms,
on two calls in a row, the second on a smaller plane; a plane too large for
the library's fixed array is refused on the host."""
import numpy as np
import pytest

from paper_2203_02479_amd import inputs

pytestmark = pytest.mark.gpu


def _conv_pair(P, seed):
    import torch
    from paper_2203_02479_amd import lar
    grid = torch.as_tensor(inputs.random_grid(P, seed, density=0.2)).cuda()
    resp = torch.as_tensor(inputs.random_spectrum(P, seed + 1)).cuda()
    ref = torch.full((P.n_wires, P.n_ticks), float("nan"), device="cuda")
    lar.fftconv(P, grid, resp, ref, lar.workspace(lar.fftconv_workspace(P)))
    got = torch.full_like(ref, float("nan"))
    lar.fftconv_noalloc(P, grid, resp, got)
    torch.cuda.synchronize()
    return got, ref


def test_noalloc_matches_workspace_call_twice():
    import torch
    from paper_2203_02479_amd import lar
    big = inputs.Plane(n_wires=800, n_ticks=6000, kind="bipolar")      # 8000 + 800 spectrum rows
    assert lar.fftconv_workspace(big) <= lar.fftconv_noalloc_max_bytes()
    for P, seed in ((big, 11), (inputs.cfg0_plane(), 12)):
        got, ref = _conv_pair(P, seed)
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), float((got - ref).abs().max())


def test_noalloc_refuses_planes_beyond_the_array():
    from paper_2203_02479_amd import lar
    P = inputs.Plane(n_wires=1000, n_ticks=16000, n_imp=10)
    assert lar.fftconv_workspace(P) > lar.fftconv_noalloc_max_bytes()
    import torch
    x = torch.zeros(1, device="cuda")
    with pytest.raises(lar.LarError) as e:
        lar.fftconv_noalloc(P, x, x, x)
    assert e.value.status == lar.LAR_ESIZE
    got, ref = _conv_pair(inputs.cfg0_plane(), 13)   # still usable after the refusal
    assert torch.equal(got, ref)
