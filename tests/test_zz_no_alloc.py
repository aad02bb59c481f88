"""The no-allocation spectrum loss (gsrf_loss_spectrum_noalloc, partial sums
in the library's fixed per-GPU scratch) against gsrf_loss_spectrum with a
caller workspace: same kernels, so results agree bit for bit, on two calls in
a row (the second smaller, over the first's leftover partial sums), on a
side stream, and the size limit is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import say
from paper_2502_01826_amd import _lib
from paper_2502_01826_amd import train as tr

pytestmark = pytest.mark.gpu


def _both(P, ne, na, lam1, lam2, c, seed, stream=None):
    sig, tgt = synth.spectra(P, ne, na, seed=seed)
    s = torch.from_numpy(sig).cuda().contiguous()
    t = torch.from_numpy(tgt).cuda().contiguous()
    ref_loss, ref_g = tr.SpectrumLoss(P, ne, na, lam1, lam2, power_scale=c)(s, t)
    loss = torch.full((P, 4), float("nan"), device="cuda")
    g = torch.full_like(s, float("nan"))
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            tr.loss_spectrum_noalloc(s, t, lam1, lam2, power_scale=c, loss=loss, grad_signal=g, stream=stream)
        torch.cuda.current_stream().wait_stream(stream)
    else:
        tr.loss_spectrum_noalloc(s, t, lam1, lam2, power_scale=c, loss=loss, grad_signal=g)
    torch.cuda.synchronize()
    return ref_loss, ref_g, loss, g


def test_noalloc_loss_matches_workspace_entry_point_twice():
    # first call: 3 spectra of 360 x 90 (216 tiles of partial sums), then a
    # ragged smaller one (2 x 37 x 70, 18 tiles) over the same scratch
    for (P, ne, na, lam1, lam2, c, seed) in [(3, 90, 360, 0.2, 0.1, 1.0, 11), (2, 37, 70, 0.3, 0.05, 1e3, 12)]:
        say("noalloc spectrum loss", P, ne, na)
        ref_loss, ref_g, loss, g = _both(P, ne, na, lam1, lam2, c, seed)
        assert torch.equal(loss, ref_loss), (loss, ref_loss)
        assert torch.equal(g, ref_g)
        assert np.isfinite(loss.cpu().numpy()).all()


def test_noalloc_loss_on_a_side_stream_and_without_gradient():
    say("noalloc spectrum loss, side stream")
    ref_loss, ref_g, loss, g = _both(1, 20, 40, 0.2, 0.1, 1.0, 13, stream=torch.cuda.Stream())
    assert torch.equal(loss, ref_loss) and torch.equal(g, ref_g)
    sig, tgt = synth.spectra(1, 20, 40, seed=13)
    s, t = torch.from_numpy(sig).cuda(), torch.from_numpy(tgt).cuda()
    l_only, none = tr.loss_spectrum_noalloc(s, t, 0.2, 0.1, want_grad=False)
    torch.cuda.synchronize()
    assert none is None and torch.equal(l_only, ref_loss)


def test_noalloc_loss_refuses_sizes_beyond_the_scratch():
    L = _lib.lib()
    # 607 spectra of 360 x 90 need 607 * 72 * 24 bytes > 1 MiB: refused on the
    # host before any pointer is touched (NULL pointers are never read)
    st = L.gsrf_loss_spectrum_noalloc(None, None, 607, 90, 360, 1.0, 0.2, 0.1, None, None, None)
    assert st == _lib.GSRF_ECAPACITY
    assert "fixed scratch" in L.gsrf_last_error().decode()
    st = L.gsrf_loss_spectrum_noalloc(None, None, 0, 90, 360, 1.0, 0.2, 0.1, None, None, None)
    assert st == _lib.GSRF_OK
