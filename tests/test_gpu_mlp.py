"""GPU checks of the learned surrogate: kernels against the FP64 network oracle.

Gradients of the training kernels are compared with the oracle that rounds
to BF16 at the same points (2e-2 relative per parameter block) and with the
plain FP64 oracle (1e-1); forward predictions and one Adam update likewise.
A small training run must cut the loss, and the projector in surrogate mode
(network where validated, exact sum elsewhere) must stay within 1e-3 of the
exact FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import rel_err
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _t(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _setup(fc, torch, n=1000, seed=0, scale=1.0):
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(3)
    s = cfg.spectral
    rng = np.random.default_rng(seed)
    M, G = s.n_mat, s.n_groups
    L = np.zeros((n, M), np.float32)
    for i in range(n):                               # a few materials per ray, realistic lengths
        k = rng.integers(1, 5)
        L[i, rng.choice(M, size=k, replace=False)] = rng.uniform(0.5, 60.0, size=k)
    Y = oracle.spectral(L, s.mu, s.phi, s.eta, s.group_of_bin, G).astype(np.float32)
    sp = fc.Spectral(_t(torch, s.mu), _t(torch, s.phi), _t(torch, s.eta), G, s.group_of_bin)
    lin = fc.fcat_mlp_linear_term(sp)
    in_scale = (1.0 / L.max(0)).astype(np.float32)
    out_scale = rng.uniform(0.2, 2.0, size=G).astype(np.float32)
    p = sg.init_params(M, G, seed) * scale
    p[-G:] = rng.normal(0, 0.05, size=G)
    sur = fc.Surrogate(params=_t(torch, p), in_scale=_t(torch, in_scale), out_scale=_t(torch, out_scale), lin=lin,
                       cell_lo=0.0, cell_hi=2.5)
    return cfg, s, L, Y, sp, sur, p, in_scale, out_scale


def _blocks(v, n_in, n_out):
    return dict(zip(["W1", "b1", "W2", "b2", "W3", "b3"], [np.ravel(a) for a in omlp.unpack(v, n_in, n_out)]))


def test_linear_term(fc):
    import torch
    cfg, s, L, Y, sp, sur, p, _, _ = _setup(fc, torch, n=64)
    ref = omlp.linear_term(s.mu, s.phi, s.eta, s.group_of_bin, s.n_groups)
    assert rel_err(sur.lin.cpu().numpy(), ref).max() <= 1e-6


@pytest.mark.parametrize("n", [64, 1000])
def test_gradients_match_oracle(fc, n):
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=n, seed=n, scale=2.0)
    M, G = s.n_mat, s.n_groups
    loss, grad = fc.fcat_mlp_gradients(sur, sp, _t(torch, L), _t(torch, Y))
    grad = grad.cpu().numpy().astype(np.float64)
    W = omlp.group_weights(s.phi, s.eta, s.group_of_bin, G)
    lin = omlp.linear_term(s.mu, s.phi, s.eta, s.group_of_bin, G)
    T = omlp.residual_targets(L, Y, W, lin)
    X = L.astype(np.float64) * in_scale
    wts = omlp.loss_weights(Y)
    l16, g16 = omlp.gradients(p, X, T, M, G, bf16=True, out_scale=osc, weights=wts)
    l64, g64 = omlp.gradients(p, X, T, M, G, out_scale=osc, weights=wts)
    assert abs(loss.item() - l16) <= 2e-3 * l16
    gb, b16, b64 = _blocks(grad, M, G), _blocks(g16, M, G), _blocks(g64, M, G)
    for k in gb:
        e16 = np.linalg.norm(gb[k] - b16[k]) / np.linalg.norm(b16[k])
        e64 = np.linalg.norm(gb[k] - b64[k]) / np.linalg.norm(b64[k])
        print(f"n={n} {k}: vs bf16 oracle {e16:.2e}, vs fp64 oracle {e64:.2e}")
        assert e16 <= 2e-2 and e64 <= 1e-1


def test_forward_matches_oracle(fc):
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=777, seed=3, scale=2.0)
    G = s.n_groups
    pred = fc.fcat_mlp_forward(sur, sp, _t(torch, L)).cpu().numpy()
    W = omlp.group_weights(s.phi, s.eta, s.group_of_bin, G)
    lin = omlp.linear_term(s.mu, s.phi, s.eta, s.group_of_bin, G)
    ref = omlp.predict_yprim(p, L, in_scale, lin, W, G, bf16=True, out_scale=osc)
    dz = np.abs(np.log(pred / ref))
    print(f"forward: max |dz| vs bf16 oracle {dz.max():.2e}")
    assert dz.max() <= 5e-5


def test_adam_step_matches_oracle(fc):
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=300, seed=5, scale=2.0)
    loss, grad = fc.fcat_mlp_gradients(sur, sp, _t(torch, L), _t(torch, Y))
    g = grad.cpu().numpy().astype(np.float64)
    params = sur.params.clone()
    tr = fc.MlpTrain(params=params, adam_m=torch.zeros_like(params), adam_v=torch.zeros_like(params), lr=1e-3)
    fc.fcat_mlp_train_step(tr, sur, sp, _t(torch, L), _t(torch, Y))
    assert tr.step == 1
    want, m, v = omlp.adam(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    np.testing.assert_allclose(params.cpu().numpy(), want, rtol=0, atol=2e-6)
    np.testing.assert_allclose(tr.adam_m.cpu().numpy(), m, rtol=1e-5, atol=1e-12)


def test_epoch_matches_separate_steps(fc):
    """Within an epoch each Adam step rewrites, in place, the BF16 views of
    the weights that the next step's gradient kernel reads; a separate
    fcat_mlp_train_step call instead builds every view afresh from the FP32
    weights.  One epoch of three batches (a ragged last one) in a shuffled
    order must therefore give bit-identical weights, Adam moments and batch
    losses to three single steps over the same samples: a view element the
    in-place rewrite missed would leave a stale weight in the later steps."""
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=1000, seed=13, scale=2.0)
    Lt, Yt = _t(torch, L), _t(torch, Y)
    order = torch.as_tensor(np.random.default_rng(13).permutation(1000).astype(np.int32), device="cuda")
    batch = 384

    def fresh():
        q = sur.params.clone()
        return fc.MlpTrain(params=q, adam_m=torch.zeros_like(q), adam_v=torch.zeros_like(q), lr=3e-3)

    ta = fresh()
    la = torch.zeros(3, dtype=torch.float32, device="cuda")
    fc.fcat_mlp_train_epoch(ta, sur, sp, Lt, Yt, order, batch, batch_loss=la)
    tb = fresh()
    lb = torch.zeros(3, dtype=torch.float32, device="cuda")
    for b, base in enumerate(range(0, 1000, batch)):
        fc.fcat_mlp_train_step(tb, sur, sp, Lt, Yt, order=order, base=base, count=min(batch, 1000 - base),
                               loss=lb[b:b + 1])
    assert ta.step == tb.step == 3
    moved = (ta.params != sur.params).float().mean().item()
    print(f"epoch vs steps: losses {la.cpu().numpy()}, share of weights moved {moved:.3f}")
    assert moved > 0.9
    for a, b in ((ta.params, tb.params), (ta.adam_m, tb.adam_m), (ta.adam_v, tb.adam_v), (la, lb)):
        assert torch.equal(a, b)


def test_setup_stats_match_oracle(fc):
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=5000, seed=7)
    G = s.n_groups
    W = omlp.group_weights(s.phi, s.eta, s.group_of_bin, G)
    lin = omlp.linear_term(s.mu, s.phi, s.eta, s.group_of_bin, G)
    i_s, o_s, tmax = fc.fcat_mlp_setup(sp, sur.lin, _t(torch, L), _t(torch, Y))
    ri, ro, rt = omlp.setup_stats(L, Y, W, lin)
    print(f"setup: in_scale {rel_err(i_s.cpu().numpy(), ri).max():.2e}, out_scale "
          f"{rel_err(o_s.cpu().numpy(), ro).max():.2e}, tau_max {abs(tmax.item() / rt - 1):.2e}")
    assert rel_err(i_s.cpu().numpy(), ri).max() <= 1e-6
    assert rel_err(o_s.cpu().numpy(), ro).max() <= 1e-3
    assert abs(tmax.item() / rt - 1) <= 1e-5


def test_validate_matches_oracle(fc):
    """Per-cell maxima and counts of the held-out validation against the oracle's
    cells and errors (network evaluated with the same BF16 split)."""
    import torch
    cfg, s, L, Y, sp, sur, p, in_scale, osc = _setup(fc, torch, n=6000, seed=11, scale=0.3)
    M, G = s.n_mat, s.n_groups
    W = omlp.group_weights(s.phi, s.eta, s.group_of_bin, G)
    lin = omlp.linear_term(s.mu, s.phi, s.eta, s.group_of_bin, G)
    mbar = omlp.mean_attenuation(W, lin)
    hi = float((L @ mbar).max()) * 0.9            # some rays beyond the range: not counted
    sur.cell_lo, sur.cell_hi = 0.0, hi
    pred = omlp.predict_yprim(p, L, in_scale, lin, W, G, bf16=True, out_scale=osc)
    e = omlp.validation_errors(pred, Y)
    c = omlp.cell_index(L, mbar, 0.0, hi, in_scale)
    ref_cnt = np.bincount(c[c >= 0], minlength=M * 16)
    ref_err = np.full(M * 16, -np.inf)
    np.maximum.at(ref_err, c[c >= 0], e[c >= 0])
    thr = float(np.median(ref_err[ref_cnt > 0]))
    err, ok, cnt = fc.fcat_mlp_validate(sur, sp, _t(torch, L), _t(torch, Y), threshold=thr, min_count=4)
    err, ok, cnt = err.cpu().numpy(), ok.cpu().numpy(), cnt.cpu().numpy()
    # cells are integer decisions from FP32 depths: allow a ray on a bin edge to land next door
    assert np.abs(cnt - ref_cnt).sum() <= 2 and cnt.sum() == pytest.approx(ref_cnt.sum(), abs=2)
    both = (cnt > 0) & (ref_cnt > 0) & (cnt == ref_cnt)
    d = np.abs(err[both] - ref_err[both])
    print(f"validate: {int((ref_cnt > 0).sum())} cells, {int(ok.sum())} ok at threshold {thr:.2e}; "
          f"max |cell error - oracle| {d.max():.2e}")
    assert np.all(d <= 1e-4 * np.maximum(1.0, ref_err[both]))
    assert np.all(np.isinf(err[cnt == 0]))
    clear = both & (np.abs(ref_err - thr) > 1e-4 * np.maximum(1.0, thr))
    want = (ref_cnt >= 4) & (ref_err <= thr)
    np.testing.assert_array_equal(ok[clear], want[clear].astype(np.uint8))


def test_training_and_surrogate_projector(fc):
    """Train on head-phantom rays (reduced size), validate, then project with the
    network where validated and the exact sum elsewhere."""
    import torch
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(5)
    pb = fc.upload(cfg)
    sur, rep = sg.build_surrogate(pb, n_samples=2_000_000, epochs=80, batch=4096, angles=np.arange(0, 720, 40),
                                  seed=11)
    print(f"training: {rep.n_train} samples, {rep.epochs} epochs, {rep.seconds:.2f} s; loss "
          f"{rep.epoch_loss[0]:.3e} -> {rep.epoch_loss[-1]:.3e}; ok cells {int(rep.cell_ok.sum())}; "
          f"held-out rays in ok cells {rep.holdout_in_ok_cells:.3f}")
    for m, (row, cnt) in enumerate(zip(rep.cell_err.reshape(-1, 16), rep.cell_count.reshape(-1, 16))):
        if cnt.sum():
            print(f"material {m}: " + " ".join("   -   " if k == 0 else f"{x:.1e}" for x, k in zip(row, cnt)))
    assert rep.epoch_loss[-1] < 0.2 * rep.epoch_loss[0]
    sur.counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    out = fc.fcat_project(pb, mode="surrogate", surrogate=sur)
    sample = [17, 500]
    o = out[sample].cpu().numpy()
    counts = sur.counts.cpu().numpy()
    del out, pb
    torch.cuda.empty_cache()
    err = rel_err(o, oracle.project(cfg, sample))
    print(f"surrogate projector: max rel err {err.max():.2e}; rays by network {counts[0]}, by exact sum {counts[1]}")
    assert counts[0] > 0 and err.max() <= 1e-3


def test_fused_surrogate_projector_matches_stage_calls(fc):
    """The surrogate projector walks, evaluates the network and sums the
    groups in one kernel.  With every cell accepted (tiny input scale, one
    optical-depth bin over everything) each ray that meets the phantom takes
    the network, so the projection of a sampled angle must equal the sum over
    groups of fcat_mlp_forward on that angle's fcat_pathlengths (the same
    walk and the same network on the stage path), and a ray that misses the
    phantom the unattenuated weight sum."""
    import torch
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(5)
    s = cfg.spectral
    M, G = s.n_mat, s.n_groups
    pb = fc.upload(cfg, scatter=False, psf=False)
    rng = np.random.default_rng(5)
    p = sg.init_params(M, G, 3)
    p[-G:] = rng.normal(0, 0.05, size=G)
    sur = fc.Surrogate(params=_t(torch, p), in_scale=_t(torch, np.full(M, 1.0 / 500.0, np.float32)),
                       out_scale=_t(torch, rng.uniform(0.2, 2.0, size=G).astype(np.float32)),
                       lin=fc.fcat_mlp_linear_term(pb.spectral), cell_ok=_t(torch, np.ones(M * 16, np.uint8)),
                       cell_lo=0.0, cell_hi=1e30, counts=torch.zeros(2, dtype=torch.int32, device="cuda"))
    out = fc.fcat_project(pb, mode="surrogate", surrogate=sur)
    n_net, n_exact = (int(x) for x in sur.counts.cpu().numpy())
    sur.counts = None
    plane = cfg.geometry.nu * cfg.geometry.nv
    w_all = float(np.sum(s.phi.astype(np.float64) * s.eta.astype(np.float64)))
    hits = 0
    for a in (0, 97, 400):
        L = fc.fcat_pathlengths(pb, M, a, a + 1).reshape(plane, M)
        yp = fc.fcat_mlp_forward(sur, pb.spectral, L).cpu().numpy().astype(np.float64)    # [G][plane]
        hit = (L.sum(1) > 0).cpu().numpy()
        hits += int(hit.sum())
        o = out[a].reshape(-1).cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(o[hit], yp.sum(0)[hit], rtol=2e-6, atol=0)
        np.testing.assert_allclose(o[~hit], w_all, rtol=2e-6)
    assert n_exact == 0 and n_net > 0.5 * cfg.geometry.n_angles * plane
    print(f"fused surrogate projector: {n_net} rays by the network, {n_exact} by the exact sum; "
          f"{hits} hit rays on the sampled angles")


def test_benchmarked_network_against_the_oracle(fc):
    """The network the benchmark reports (head workload, 4M pairs with 10%
    held out, 120 epochs, the build_surrogate defaults) projects within 1e-3
    of the FP64 oracle on sampled angles, with the network taking most of the
    hit rays."""
    import torch
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(5)
    pb = fc.upload(cfg)
    sur, rep = sg.build_surrogate(pb, n_samples=4_000_000, epochs=120)
    assert rep.n_train + rep.n_holdout == 4_000_000 and rep.epochs == 120
    sur.counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    out = fc.fcat_project(pb, mode="surrogate", surrogate=sur)
    sample = [0, 251, 611]
    o = out[sample].cpu().numpy()
    counts = sur.counts.cpu().numpy()
    del out, pb
    torch.cuda.empty_cache()
    err = rel_err(o, oracle.project(cfg, sample))
    share = counts[0] / max(counts[0] + counts[1], 1)
    print(f"benchmarked network: max rel err {err.max():.2e}, rms {np.sqrt((err ** 2).mean()):.2e}; "
          f"network share of hit rays {share:.3f}")
    assert err.max() <= 1e-3 and share > 0.5


def test_training_resumes_from_a_checkpoint(fc, tmp_path):
    """Two epochs, a checkpoint, then a resumed call for the other two give
    the same weights, Adam state and loss history as four epochs in one go."""
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(1)
    pb = fc.upload(cfg)
    kw = dict(n_samples=20000, epochs=4, batch=1024, angles=np.arange(0, 45, 3), seed=5)
    sur_a, rep_a = sg.build_surrogate(pb, **kw)
    ck = str(tmp_path / "surrogate.npz")
    _, rep_half = sg.build_surrogate(pb, checkpoint=ck, stop_after=2, **kw)
    assert len(rep_half.epoch_loss) == 2
    sur_b, rep_b = sg.build_surrogate(pb, checkpoint=ck, resume=True, **kw)
    np.testing.assert_array_equal(sur_b.params.cpu().numpy(), sur_a.params.cpu().numpy())
    assert rep_b.epoch_loss == rep_a.epoch_loss
    np.testing.assert_array_equal(rep_b.cell_ok, rep_a.cell_ok)
    with np.load(ck, allow_pickle=False) as z:
        assert int(z["epoch"]) == 3 and int(z["step"]) > 0


def test_stage_timer_counts_one_walk_launch_per_chunk(fc):
    """The benchmark divides the walk stage's time by its launch count: every
    mode must record exactly one walk launch per angle chunk, a surrogate
    call with ray counts included (its count total is set-up work), and the
    counts must cover every valid ray of the detector."""
    import torch
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(2)                     # with a PSF: group signals pass through angle chunks
    s = cfg.spectral
    M, G = s.n_mat, s.n_groups
    pb = fc.upload(cfg)
    rng = np.random.default_rng(8)
    p = sg.init_params(M, G, 2)
    sur = fc.Surrogate(params=_t(torch, p), in_scale=_t(torch, np.full(M, 1.0 / 500.0, np.float32)),
                       out_scale=_t(torch, rng.uniform(0.2, 2.0, size=G).astype(np.float32)),
                       lin=fc.fcat_mlp_linear_term(pb.spectral), cell_ok=_t(torch, np.ones(M * 16, np.uint8)),
                       cell_lo=0.0, cell_hi=1e30, counts=torch.zeros(2, dtype=torch.int32, device="cuda"))
    A = cfg.geometry.n_angles
    chunk = 100                                    # 360 angles: three chunks of 100 and one of 60
    fc.fcat_timing_enable(True)
    try:
        for mode in ("plain", "split_bf16", "surrogate"):
            fc.fcat_timing_read(reset=True)
            fc.fcat_project(pb, mode=mode, surrogate=sur if mode == "surrogate" else None, angles_per_chunk=chunk)
            torch.cuda.synchronize()
            st = fc.fcat_timing_read(reset=True)
            assert st["trace"][1] == -(-A // chunk), (mode, st)
    finally:
        fc.fcat_timing_enable(False)
    n_net, n_exact = (int(x) for x in sur.counts.cpu().numpy())
    print(f"{A} angles in chunks of {chunk}: rays by the network {n_net}, by the exact sum {n_exact}")
    assert n_exact == 0 and 0 < n_net <= A * cfg.geometry.nu * cfg.geometry.nv
    del pb
    torch.cuda.empty_cache()
