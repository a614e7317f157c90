"""Learned sub-sample TDoA on the GPU: the hand-written MLP kernels against the
FP64 oracle (forward, gradient, Adam), and a trained network against FCC and
GCC-PHAT with quadratic interpolation on held-out fractional-delay frames."""
import math

import numpy as np
import pytest

import oracle.fcc_oracle as O
import oracle.mlp_oracle as MO
from gen import fractional_delay_frames, circular_array

pytestmark = pytest.mark.gpu

# unit roundoff of FP16 operands; a product of two rounded operands is off by
# at most (1 + u)^2 - 1 < 2.001 u relative
U16 = 2.0 ** -11
GAMMA = 2.001 * U16
GELU_SLOPE = 1.13       # max |gelu'(x)| of the tanh form (attained near x = 2.4)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


@pytest.fixture(scope="module")
def learned(torch):
    import paper_2204_13622_amd.learned as L
    return L


def _theta(in_dim, H, seed, clip_side=0, coef=None):
    """Oracle initialisation with random hidden biases.  With clip_side = +-1
    the log-variance bias puts the clip in the widest gap between the sorted
    raw log-variances of the middle third of `coef`'s rows, so a third to two
    thirds of the rows are clipped and no row sits near the boundary, where
    FP16 rounding could move it across."""
    theta = MO.init_params(in_dim, H, seed)
    rng = np.random.default_rng(seed + 1)
    W1, b1, W2, b2, W3, b3v = MO.unpack(theta, in_dim, H)
    b1[:] = 0.1 * rng.standard_normal(H)
    b2[:] = 0.1 * rng.standard_normal(H)
    if clip_side:
        s_raw = MO.forward(theta, coef.astype(np.float64), H)[2][5]
        srt = np.sort(s_raw)
        lo, hi = len(srt) // 3, 2 * len(srt) // 3
        k = lo + int(np.argmax(np.diff(srt[lo:hi + 1])))
        b3v[:] = (0.3, clip_side * MO.S_CLIP - 0.5 * (srt[k] + srt[k + 1]))
    return theta.astype(np.float32).astype(np.float64)


def _coef(rows, in_dim, seed):
    c = np.random.default_rng(seed).standard_normal((rows, in_dim)).astype(np.float32)
    c[rows // 3] = 0.0          # a silent pair-frame: features stay zero
    return c


def _forward_bound(theta, coef, H):
    """First-order bound on |o_gpu - o_exact| when every matrix operand is
    rounded to FP16 and accumulated in FP32 (FP32 terms are negligible)."""
    u, z1, h1, z2, h2, _ = MO.forward(theta, coef, H)[2]
    W1, b1, W2, b2, W3, b3 = MO.unpack(theta, u.shape[1], H)
    e1 = GAMMA * (np.abs(u) @ np.abs(W1))
    eh1 = GELU_SLOPE * e1
    e2 = GAMMA * (np.abs(h1) @ np.abs(W2)) + eh1 @ np.abs(W2)
    eh2 = GELU_SLOPE * e2
    return GAMMA * (np.abs(h2) @ np.abs(W3)) + eh2 @ np.abs(W3)


@pytest.mark.parametrize("in_dim,H,rows", [(10, 128, 300), (22, 128, 1000), (18, 48, 77), (64, 512, 130),
                                         (10, 32, 100), (40, 64, 333), (64, 128, 17),
                                         (10, 128, 1), (22, 64, 16), (18, 48, 1)])   # one row; one tile
def test_forward_matches_oracle(torch, learned, in_dim, H, rows):
    theta = _theta(in_dim, H, 10 + in_dim)
    coef = _coef(rows, in_dim, 20 + rows)
    net = learned.Mlp(in_dim, H, params=theta)
    out = net.forward(torch.from_numpy(coef).cuda()).cpu().numpy().astype(np.float64)
    mu, s, _ = MO.forward(theta, coef.astype(np.float64), H)
    bound = _forward_bound(theta, coef.astype(np.float64), H)
    err = np.abs(out - np.stack([mu, s], 1))
    assert np.all(err <= 1.5 * bound + 1e-5), (err / (bound + 1e-12)).max()
    assert np.all(out[rows // 3] == out[rows // 3])        # zero row stays finite


@pytest.mark.parametrize("in_dim,H,rows,clip_side", [(10, 128, 300, 0), (22, 128, 160, 1), (18, 48, 77, -1)])
def test_gradient_matches_oracle(torch, learned, in_dim, H, rows, clip_side):
    coef = _coef(rows, in_dim, 40 + rows)
    theta = _theta(in_dim, H, 30 + in_dim, clip_side, coef)
    target = np.random.default_rng(rows).uniform(-4.0, 4.0, rows).astype(np.float32)
    net = learned.Mlp(in_dim, H, params=theta)
    loss, out = net.loss_and_grad(torch.from_numpy(coef).cuda(), torch.from_numpy(target).cuda())
    g = net.grad.cpu().numpy().astype(np.float64)
    L_ref, g_ref = MO.loss_and_grad(theta, coef.astype(np.float64), target.astype(np.float64), H)
    _, s_ref, cache = MO.forward(theta, coef.astype(np.float64), H)
    clipped = np.abs(cache[5]) >= MO.S_CLIP
    if clip_side:
        assert rows // 4 < clipped.sum() < 3 * rows // 4     # both branches of the clip are exercised
        # no row within 2e-3 of the clip: emulating the FP16 operand rounding
        # in FP64 moves these raw log-variances by at most 3e-4
        assert np.abs(np.abs(cache[5]) - MO.S_CLIP).min() > 2e-3
    assert abs(float(loss.item()) - L_ref) <= 2e-3 * max(1.0, abs(L_ref))
    # every gradient passes through at most five FP16-rounded products; the
    # blockwise error relative to the block's norm stays within ~10 GAMMA kappa
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    sizes = [in_dim * H, H, H * H, H, 2 * H, 2]
    o = 0
    for name, n in zip(names, sizes):
        ref, got = g_ref[o:o + n], g[o:o + n]
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel < 1e-2, (name, rel)
        o += n


def test_adam_matches_oracle(torch, learned):
    in_dim, H = 10, 32
    n = MO.num_params(in_dim, H)
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(n).astype(np.float32)
    net = learned.Mlp(in_dim, H, params=theta)
    th, m, v = theta.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(lr=1e-2)
        th, m, v = MO.adam_step(th, m, v, g.astype(np.float64), step, 1e-2)
    got = net.params.cpu().numpy()
    assert np.abs(got - th).max() < 1e-5


def _cfg5_data(torch, fcc, seed, frames, rank, **gen):
    x, d, xyz = fractional_delay_frames(seed, frames, **gen)
    plan = fcc.Plan(xyz, 16000.0, frame_size=512, hop=512, rank=rank)
    spec = plan.spectra(torch.from_numpy(x).cuda())
    pairs = np.array(O.mic_pairs(8))
    target = (d[:, pairs[:, 0]] - d[:, pairs[:, 1]]).astype(np.float32)
    return plan, spec, x, target


# the learned-stage workload: 1e6 training and 1e5 held-out pair-frames
# (8 microphones, 28 pairs per frame)
TRAIN_FRAMES = 35715                  # 1,000,020 pair-frames
EVAL_FRAMES = 3572                    # 100,016 pair-frames
# a shifted split: reverberant frames (RT60 20-60 ms, DRR 0-10 dB) at SNR
# -5 .. 20 dB, outside the training distribution
STRESS = dict(rt60=(0.02, 0.06), snr_db=(-5.0, 20.0))


def _evaluate(learned, plan, spec, net, thr):
    tau, conf = learned.tdoa_learned(plan, spec, net, thr)
    mlp, _ = learned.tdoa_learned(plan, spec, net, 0.0)
    par = plan.tdoa_parabolic(spec).cpu().numpy()
    return tau.cpu().numpy(), conf.cpu().numpy(), mlp.cpu().numpy(), par


def test_learned_beats_interpolated_fcc_and_gcc(torch, learned):
    """Trained on 1e6 fractional-delay pair-frames on the GPU (the project's
    FP16 forward / backward / Adam kernels), the confidence threshold chosen
    on 1e5 validation pair-frames, scored on 1e5 held-out pair-frames against
    interpolated FCC (GPU and FP64) and FP64 GCC-PHAT with quadratic
    interpolation (Sec. 2), the fallback and the judge.  A shifted split
    (reverberant, lower SNR) picks its own threshold, where the fallback can
    take over from a network that has not seen such frames."""
    import paper_2204_13622_amd as fcc
    rank = 5
    plan, spec_tr, _, t_tr = _cfg5_data(torch, fcc, 51, TRAIN_FRAMES, rank)
    _, spec_va, _, t_va = _cfg5_data(torch, fcc, 52, EVAL_FRAMES, rank)
    _, spec_te, x_te, t_te = _cfg5_data(torch, fcc, 53, EVAL_FRAMES, rank)
    assert plan.tau_max == 4 and plan.P == 28
    assert TRAIN_FRAMES * plan.P >= 1_000_000 and EVAL_FRAMES * plan.P >= 100_000
    coef_tr = plan.coefficients(spec_tr)
    net = learned.Mlp(2 * rank, 128, seed=7)
    hist = net.fit(coef_tr, torch.from_numpy(t_tr).cuda(), epochs=8, batch=2048, lr=2e-3)
    print("epoch losses", [round(h, 4) for h in hist], flush=True)
    assert all(math.isfinite(h) for h in hist) and hist[-1] < hist[0]
    del coef_tr, spec_tr

    # threshold from the validation split
    mu_va = net.forward(plan.coefficients(spec_va))[..., 0].cpu().numpy()
    tau_va, conf_va, mlp_va, par_va = _evaluate(learned, plan, spec_va, net, 0.0)
    assert np.array_equal(tau_va, mu_va)                    # threshold 0: the network alone
    thr = learned.choose_threshold(mlp_va, conf_va, par_va, t_va)

    # held-out split
    tau, conf, net_only, par = _evaluate(learned, plan, spec_te, net, thr)
    fallback, _ = learned.tdoa_learned(plan, spec_te, net, math.inf)
    assert np.array_equal(fallback.cpu().numpy(), par)     # threshold +inf: plain FCC + interpolation
    Rh = O.pipeline_spectra(x_te.astype(np.float64), 512, 512)
    gcc_par = O.tdoa_parabolic_from_corr(O.gcc_corr(Rh, 512, 4), 4)
    fcc_par = O.tdoa_parabolic_from_corr(O.fcc_corr(Rh, O.fcc_basis(512, 4, rank)), 4)
    mae = {k: float(np.abs(v - t_te).mean()) for k, v in
           [("learned", tau), ("mlp_only", net_only), ("fcc_parabolic_gpu", par),
            ("fcc_parabolic_fp64", fcc_par), ("gcc_parabolic_fp64", gcc_par)]}
    share = float((conf < thr).mean())
    print(f"held-out MAE (samples) over {t_te.size} pair-frames: {mae}, threshold {thr}, "
          f"fallback share {share:.4f}", flush=True)
    # the GPU's interpolated FCC lag is the FP64 one up to FP32 rounding
    assert abs(mae["fcc_parabolic_gpu"] - mae["fcc_parabolic_fp64"]) < 1e-3
    assert mae["learned"] < 0.6 * mae["fcc_parabolic_gpu"]
    assert mae["learned"] < 0.6 * mae["gcc_parabolic_fp64"]
    assert mae["learned"] <= 1.05 * mae["mlp_only"]
    # the confidence ranks the network's own errors: its least confident tenth
    # errs far more than its most confident tenth
    err = np.abs(net_only - t_te).ravel()
    order = np.argsort(conf.ravel())
    tenth = order.size // 10
    lo, hi = err[order[:tenth]].mean(), err[order[-tenth:]].mean()
    print(f"MLP MAE, least / most confident tenth: {lo:.4f} / {hi:.4f}", flush=True)
    assert lo > 3.0 * hi

    # shifted split: its own validation picks the threshold
    _, spec_sv, _, t_sv = _cfg5_data(torch, fcc, 54, EVAL_FRAMES, rank, **STRESS)
    _, spec_st, _, t_st = _cfg5_data(torch, fcc, 55, EVAL_FRAMES, rank, **STRESS)
    _, conf_sv, mlp_sv, par_sv = _evaluate(learned, plan, spec_sv, net, 0.0)
    thr_s = learned.choose_threshold(mlp_sv, conf_sv, par_sv, t_sv)
    tau_s, conf_s, mlp_s, par_s = _evaluate(learned, plan, spec_st, net, thr_s)
    mae_s = {k: float(np.abs(v - t_st).mean()) for k, v in
             [("learned", tau_s), ("mlp_only", mlp_s), ("fcc_parabolic_gpu", par_s)]}
    share_s = float((conf_s < thr_s).mean())
    print(f"shifted held-out MAE: {mae_s}, threshold {thr_s}, fallback share {share_s:.4f}", flush=True)
    assert mae_s["learned"] <= 1.02 * min(mae_s["mlp_only"], mae_s["fcc_parabolic_gpu"])


def test_learned_entry_errors(torch, learned):
    import paper_2204_13622_amd as fcc
    plan = fcc.Plan(circular_array(8, 0.04), 16000.0, frame_size=512, hop=512, rank=5)
    spec = plan.spectra(torch.zeros((8, 512 * 3), dtype=torch.float32, device="cuda"))
    net = learned.Mlp(10, 128)
    empty = spec[:0]
    tau, conf = learned.tdoa_learned(plan, empty, net, 1.0)
    assert tau.shape == (0, 28)
    tau, conf = learned.tdoa_learned(plan, spec, net, 1.0)     # silent frames: zero coefficients
    assert np.all(np.isfinite(tau.cpu().numpy()))
    with pytest.raises(ValueError):
        learned.tdoa_learned(plan, spec, learned.Mlp(12, 128), 1.0)
    with pytest.raises(fcc.FccError):
        learned.Mlp(10, 40).forward(torch.zeros((4, 10), device="cuda"))
