"""GPU parity of the training steps (losses, SGD) against the FP64 oracle,
through the C ABI, and a first-order check of a whole training iteration."""
import numpy as np
import pytest
import torch

import synth
from oracle import train_oracle as to
from gpu_common import gpu_problem, say
from paper_2502_01826_amd import train as tr

pytestmark = pytest.mark.gpu

LOSS_RTOL = 1e-4      # loss values (FP32 sums of FP32 terms vs FP64)
GRAD_RTOL = 1e-4      # per-pixel gradient, relative to the largest |G| of the pair


def _gpu_spectrum_loss(sig, tgt, lam1, lam2, pscale=1.0):
    P, ne, na = tgt.shape
    fn = tr.SpectrumLoss(P, ne, na, lam1, lam2, power_scale=pscale)
    s = torch.from_numpy(sig).cuda().contiguous()
    t = torch.from_numpy(tgt).cuda().contiguous()
    loss, g = fn(s, t)
    loss2, g2 = fn(s, t)
    torch.cuda.synchronize()
    assert torch.equal(loss, loss2) and torch.equal(g, g2)        # deterministic
    return loss.cpu().numpy().astype(np.float64), torch.view_as_complex(g).cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("P,ne,na,lam1,lam2,c", [(2, 37, 70, 0.2, 0.1, 1.0), (1, 16, 32, 0.0, 0.0, 1.0),
                                                  (1, 9, 36, 1.0, 0.0, 1.0), (3, 5, 7, 0.0, 1.0, 1.0),
                                                  (1, 90, 360, 0.2, 0.05, 1.0), (2, 40, 50, 0.3, 0.02, 1e4)])
def test_spectrum_loss_matches_oracle(P, ne, na, lam1, lam2, c):
    """Several 16 x 32 tiles with ragged last row and column (37 x 70), one exact
    tile, spectra smaller than the SSIM window (5 x 7), the 360 x 90 grid, and
    rays 100x weaker than the target scale (power_scale 1e4)."""
    say("spectrum loss", P, ne, na, lam1, lam2, c)
    sig, tgt = synth.spectra(P, ne, na, seed=ne * 1000 + na)
    sig = (sig / np.sqrt(c)).astype(np.float32)
    loss, G = _gpu_spectrum_loss(sig, tgt, lam1, lam2, c)
    for k in range(P):
        ref = to.spectrum_loss_terms(sig[k, ..., 0] + 1j * sig[k, ..., 1], tgt[k], lam1, lam2, power_scale=c)
        want = np.array([ref["total"], ref["l1"], ref["ssim_loss"], ref["fourier"]])
        assert np.all(np.abs(loss[k] - want) <= LOSS_RTOL * np.maximum(np.abs(want), 1e-6)), (k, loss[k], want)
        err = np.abs(G[k] - ref["G"]).max()
        assert err <= GRAD_RTOL * np.abs(ref["G"]).max(), (k, err, np.abs(ref["G"]).max())


def test_spectrum_loss_without_gradient_and_empty_batch():
    sig, tgt = synth.spectra(1, 20, 40, seed=3)
    fn = tr.SpectrumLoss(1, 20, 40, 0.2, 0.1)
    s, t = torch.from_numpy(sig).cuda(), torch.from_numpy(tgt).cuda()
    l_only, none = fn(s, t, want_grad=False)
    l_both, _ = fn(s, t)
    torch.cuda.synchronize()
    assert none is None and torch.equal(l_only, l_both)
    e = tr.SpectrumLoss(0, 20, 40, 0.2, 0.1)
    z = torch.zeros((0, 20, 40, 2), device="cuda")
    loss, g = e(z, torch.zeros((0, 20, 40), device="cuda"))
    assert loss.shape == (0, 4) and g.shape == (0, 20, 40, 2)


def test_single_antenna_losses_match_oracle():
    rng = np.random.default_rng(21)
    P = 300
    s = rng.normal(0, 0.3, (P, 2)).astype(np.float32)
    s[7] = 0.0                                                   # S_hat = 0: +inf loss, zero gradient
    t_db = rng.normal(-20, 5, P).astype(np.float32)
    t_c = rng.normal(0, 0.3, (P, 2)).astype(np.float32)
    sd = torch.from_numpy(s).cuda()
    l_db, g_db = tr.loss_single(sd, torch.from_numpy(t_db).cuda(), tr.RSSI_DB)
    l_c, g_c = tr.loss_single(sd, torch.from_numpy(t_c).cuda(), tr.COMPLEX_L2)
    torch.cuda.synchronize()
    l_db, g_db, l_c, g_c = (x.cpu().numpy() for x in (l_db, g_db, l_c, g_c))
    for k in range(P):
        sk = complex(s[k, 0], s[k, 1])
        rc = to.single_loss_terms(sk, complex(t_c[k, 0], t_c[k, 1]), "complex")
        assert abs(l_c[k] - rc["loss"]) <= 1e-6 * max(rc["loss"], 1e-30)
        assert abs(complex(*g_c[k]) - rc["G"]) <= 1e-6 * abs(rc["G"]) + 1e-30
        if k == 7:
            assert np.isinf(l_db[k]) and l_db[k] > 0 and np.all(g_db[k] == 0)
            continue
        rd = to.single_loss_terms(sk, float(t_db[k]), "rssi")
        assert abs(l_db[k] - rd["loss"]) <= 1e-6 * max(rd["loss"], 1.0)
        assert abs(complex(*g_db[k]) - rd["G"]) <= 1e-6 * abs(rd["G"])


@pytest.mark.parametrize("iteration", [0, 1234, 30_000, 45_000])
def test_sgd_step_is_bit_exact(iteration):
    rng = np.random.default_rng([22, iteration])
    G, K = 1003, 9
    shapes = dict(means=(G, 3), log_scales=(G, 3), quats=(G, 4), logits=(G,), coeffs=(G, K, 2))
    p = {k: rng.normal(0, 1, s).astype(np.float32) for k, s in shapes.items()}
    g = {k: rng.normal(0, 10, s).astype(np.float32) for k, s in shapes.items()}
    pd = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
    gd = {k: torch.from_numpy(v).cuda() for k, v in g.items()}
    tr.sgd_step(pd, gd, iteration, fle_L=2)
    torch.cuda.synchronize()
    want = to.sgd_step(p, g, iteration)
    for k in shapes:
        assert np.array_equal(pd[k].cpu().numpy().view(np.uint32), want[k].view(np.uint32)), k


def test_sgd_custom_rates_no_decay_and_unaligned_arrays():
    rng = np.random.default_rng(23)
    G = 64
    p = {k: rng.normal(0, 1, s).astype(np.float32) for k, s in
         dict(means=(G, 3), log_scales=(G, 3), quats=(G, 4), logits=(G,), coeffs=(G, 1, 2)).items()}
    g = {k: rng.normal(0, 1, v.shape).astype(np.float32) for k, v in p.items()}
    lr = tr.LearningRates(mean_init=0.3, mean_final=0.3, mean_steps=0, log_scale=0.1, quat=0.0, logit=1.0,
                          coeff=0.5)
    def offset(v):      # a view starting 4 bytes into its buffer: the kernel's scalar path
        buf = torch.zeros(v.size + 1, dtype=torch.float32, device="cuda")
        buf[1:] = torch.from_numpy(v.ravel()).cuda()
        return buf[1:].view(v.shape)

    pd = {k: offset(v) for k, v in p.items()}
    tr.sgd_step(pd, {k: torch.from_numpy(v).cuda() for k, v in g.items()}, 99, fle_L=0, lr=lr)
    torch.cuda.synchronize()
    want = to.sgd_step(p, g, 99, dict(mean_init=0.3, mean_final=0.3, mean_steps=0, log_scale=0.1, quat=0.0,
                                      logit=1.0, coeff=0.5))
    for k in p:
        assert np.array_equal(pd[k].cpu().numpy().view(np.uint32), want[k].view(np.uint32)), k
    assert np.array_equal(pd["quats"].cpu().numpy(), p["quats"])          # zero rate leaves the attribute


def test_training_iteration_descends():
    """render -> spectrum loss -> adjoint -> SGD-style step on the tiny room: a
    small step along the computed coefficient gradient lowers the loss by about
    eta |g|^2 (first order), which checks the sign and scale conventions from
    the loss through the adjoint end to end."""
    b = synth.tiny(n=1500)
    g = b.grid
    sc = b.scenes[0]
    rng = np.random.default_rng(24)
    # target: the power spectrum of the same room with perturbed radiance
    tcoef = (sc.coeffs + rng.normal(0, 0.05, sc.coeffs.shape)).astype(np.float32)
    tb = synth.Batch([synth.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, tcoef)], b.pairs, g)
    tsig, _, _ = gpu_problem(tb).forward()
    target = (tsig ** 2).sum(-1)
    c = 1.0 / float(target.max())                         # spectra normalised to a peak of 1
    target = (target * c).contiguous()
    prob = gpu_problem(b)
    fn = tr.SpectrumLoss(1, g.n_el, g.n_az, 0.2, 0.1, power_scale=c)

    def loss_of():
        s, _, _ = prob.forward()
        l, G = fn(s, target)
        return s, float(l[0, 0]), G

    s, l0, G = loss_of()
    grads = prob.render_bwd(s.contiguous(), G)
    gc = grads[4].clone()
    g2 = float((gc.double() ** 2).sum())
    eta = 1e-3 * l0 / g2
    prob.coeffs.sub_(eta * gc)
    _, l1, _ = loss_of()
    torch.cuda.synchronize()
    drop = l0 - l1
    say(f"loss {l0:.6e} -> {l1:.6e}, predicted drop {eta * g2:.3e}, got {drop:.3e}")
    assert 0.5 * eta * g2 < drop < 1.5 * eta * g2
