"""The GPU discrete adjoint (through the C ABI) against the oracle's forward
sensitivities of the same frozen-schedule replay: the replayed end state,
the per-cell vector-Jacobian products, the autograd wrapper, and the failure
paths."""
import numpy as np
import pytest

from paper_2312_02836_amd import synth
from tests.parity import assert_parity, gate_for

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-6, 1e-10


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2312_02836_amd import burn as B
    return B


def _cot(spec, C, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(spec.n_species, C)), rng.normal(size=C)


def _run_gpu(B, spec, cells, t_end, gY, gE, log_mult=None, max_steps=2048):
    import torch
    net = B.Network(spec)
    run = B.AdjointRun(net, cells.Y, cells.rho, cells.T, t_end, RTOL, ATOL, log_mult,
                       max_steps=max_steps)
    Y, T, E, st = run.forward()
    grad = run.backward(gY, gE)
    torch.cuda.synchronize()
    out = (Y.cpu().numpy(), T.cpu().numpy(), E.cpu().numpy(), st.cpu().numpy(),
           run.counters.cpu().numpy(), grad.cpu().numpy())
    net.close()
    return out


# Per-cell gradients agree with the oracle's to this share of the cell's
# largest component (observed 1-2e-11 on the 13/30 and 21/60 networks).
GRAD_RTOL = 1e-10


def _check_adjoint(B, oracle, spec, cells, t_end, seed=0, log_mult=None, grad_rtol=GRAD_RTOL):
    C = cells.n_cells
    gY, gE = _cot(spec, C, seed)
    Yg, Tg, Eg, stg, cntg, gg = _run_gpu(B, spec, cells, t_end, gY, gE, log_mult)
    onet = oracle.OracleNet(spec)
    Yo, To, sto, cnto, S, unc = oracle.sens(onet, cells, t_end, RTOL, ATOL, log_mult=log_mult)

    def tight(idx):
        r = oracle.burn(onet, cells.subset(idx), t_end, RTOL * 1e-4, ATOL * 1e-4,
                        log_mult=log_mult)
        return r[0], r[1]

    # the replayed end state
    rep = assert_parity((Yg, Tg, stg, cntg), (Yo, To, sto, cnto), RTOL, ATOL, tight=tight,
                        **gate_for(spec))
    assert np.allclose(Eg, spec.c_v * (Tg - cells.T), rtol=1e-12, atol=1e-14)
    # gradients where both sides replayed the same schedule
    go = oracle.vjp(onet, S, gY, gE)
    same = rep["same_counters"] & (sto == 0)
    scale = np.abs(go).max(axis=0)
    err = np.abs(gg - go).max(axis=0)
    bad = np.nonzero(same & (err > grad_rtol * scale + 1e-300))[0]
    print(f"adjoint: cells {C}, same schedule {int(same.sum())}, max rel grad err "
          f"{(err[same] / np.maximum(scale[same], 1e-300)).max():.3e}", flush=True)
    assert bad.size == 0, (bad[:10], err[bad[:10]], scale[bad[:10]])
    assert np.all(gg[:, sto != 0] == 0.0)
    return gg, go


def test_adjoint_synth21(gpu, oracle):
    """The 21-species / 60-reaction sensitivity workload, 261 cells (a
    ragged last workgroup)."""
    cfg = synth.config(5, n_cells=261)
    _check_adjoint(gpu, oracle, cfg.networks[0], cfg.cells[0], cfg.t_end)


@pytest.mark.parametrize("which", [(5, 0, 261), (4, 3, 33)])
def test_adjoint_state_pool_bitwise(gpu, which):
    """The corrected states the replay keeps in the workspace's pool are the
    doubles the reverse sweep would recompute from checkpoints: end state,
    E and gradients are bitwise the same with no pool, a pool for part of
    the cells and a pool for all of them (and the pool grows to fit on a
    second forward call).  21/60 network (two cells per wave) and 50/150
    (one cell per wave)."""
    import torch
    cfg_n, item, C = which
    cfg = synth.config(cfg_n, n_cells=C)
    spec, cells = cfg.networks[item], cfg.cells[item]
    gY, gE = _cot(spec, C, 3)
    net = gpu.Network(spec)
    outs, pools = [], []
    for steps in (None, "half", "all", "grow"):
        if steps in ("half", "all"):
            total = outs[0][-1]
            steps = total // 2 if steps == "half" else total
        run = gpu.AdjointRun(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL,
                             max_steps=2048, states_steps=None if steps == "grow" else steps)
        if steps == "grow":
            run.forward()
            run.backward(gY, gE)
        Y, T, E, st = run.forward()
        g = run.backward(gY, gE)
        torch.cuda.synchronize()
        pools.append(run.pool_steps)
        outs.append((Y.cpu().numpy(), T.cpu().numpy(), E.cpu().numpy(), st.cpu().numpy(),
                     g.cpu().numpy(), run.recorded_steps()))
    net.close()
    assert pools[0] == 0 and 0 < pools[1] < pools[2] and pools[3] >= pools[2]
    assert np.all(outs[0][3] == 0)
    for o in outs[1:]:
        for a, b in zip(o[:5], outs[0][:5]):
            assert np.array_equal(a, b)


def test_adjoint_synth13_with_multipliers(gpu, oracle):
    cfg = synth.config(2, n_cells=130)
    lm = np.random.default_rng(7).normal(0.0, 0.3, cfg.networks[0].n_reactions)
    _check_adjoint(gpu, oracle, cfg.networks[0], cfg.cells[0], cfg.t_end, seed=1, log_mult=lm)


def test_adjoint_synth50(gpu, oracle):
    """50 species / 150 reactions: one cell per wave with n = 51 lanes.  This
    network's Newton matrices are ill-conditioned enough that the rounding
    differences of the two replays' corrected states (each solved to 1e-10 in
    the weighted norm, by different iterations) show in the gradients at
    ~6e-9 of their scale; the bound is 1e-8."""
    cfg = synth.config(4, n_cells=33)
    _check_adjoint(gpu, oracle, cfg.networks[3], cfg.cells[3], cfg.t_end, seed=2,
                   grad_rtol=1e-8)


def test_adjoint_bateman_chain(gpu, oracle):
    """A -> B -> C with heat at tight tolerance: the GPU gradients against the
    closed-form d(A, B, C, T)/d ln k contracted with the cotangents."""
    k1, k2, q1, q2, cv = 3.0, 0.7, 1.5, 2.5, 10.0
    spec = synth.chain_network([k1, k2], q=[q1, q2], c_v=cv)
    cells = synth.Cells(np.array([[1.0], [0.0], [0.0]]), np.array([1.0]), np.array([2.0]))
    gY, gE = np.array([[0.3], [-1.2], [0.7]]), np.array([0.5])
    import torch
    net = gpu.Network(spec)
    run = gpu.AdjointRun(net, cells.Y, cells.rho, cells.T, 2.0, 1e-10, 1e-14)
    run.forward()
    g = run.backward(gY, gE).cpu().numpy()[:, 0]
    t = 2.0
    e1, e2 = np.exp(-k1 * t), np.exp(-k2 * t)
    dA = np.array([-k1 * t * e1, 0.0])
    dB = np.array([k1 * (k2 / (k2 - k1) ** 2 * (e1 - e2) - k1 / (k2 - k1) * t * e1),
                   k2 * (-k1 / (k2 - k1) ** 2 * (e1 - e2) + k1 / (k2 - k1) * t * e2)])
    dC = -dA - dB
    dE = -q1 * dA + q2 * dC  # E = c_v dT
    ref = gY[0, 0] * dA + gY[1, 0] * dB + gY[2, 0] * dC + gE[0] * dE
    assert np.allclose(g, ref, rtol=1e-6, atol=1e-9), (g, ref)
    net.close()


def test_autograd_function(gpu, oracle):
    import torch
    cfg = synth.config(5, n_cells=64)
    spec, cells = cfg.networks[0], cfg.cells[0]
    net = gpu.Network(spec)
    dev = torch.device("cuda", 0)
    p = torch.zeros(spec.n_reactions, dtype=torch.float64, device=dev, requires_grad=True)
    Y, E, st = gpu.BurnFn.apply(p, net, cells.Y, cells.rho, cells.T, cfg.t_end)
    w = torch.linspace(0.5, 1.5, spec.n_species, dtype=torch.float64, device=dev)
    loss = (w[:, None] * Y).sum() + 0.1 * E.sum()
    loss.backward()
    gY = np.broadcast_to(np.linspace(0.5, 1.5, spec.n_species)[:, None], (spec.n_species, 64))
    onet = oracle.OracleNet(spec)
    Yo, To, sto, cnto, S, unc = oracle.sens(onet, cells, cfg.t_end)
    go = oracle.vjp(onet, S, gY, np.full(64, 0.1)).sum(axis=1)
    gg = p.grad.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    # summed over cells: a few cells may have taken another schedule, so the
    # bound is on the scale of the whole gradient
    assert np.allclose(gg, go, rtol=0, atol=1e-6 * np.abs(go).max()), np.abs(gg - go).max()
    net.close()


def test_adjoint_failure_paths(gpu, oracle):
    cfg = synth.config(5, n_cells=20)
    spec, cells = cfg.networks[0], cfg.cells[0]
    bad = synth.Cells(cells.Y.copy(), cells.rho.copy(), cells.T.copy())
    bad.rho[3] = np.nan
    bad.T[5] = -1.0
    gY, gE = _cot(spec, 20, 4)
    Yg, Tg, Eg, stg, cntg, gg = _run_gpu(gpu, spec, bad, cfg.t_end, gY, gE)
    assert stg[3] == 4 and stg[5] == 4
    assert np.all(gg[:, [3, 5]] == 0.0) and np.all(Eg[[3, 5]] == 0.0)
    ok = np.setdiff1d(np.arange(20), [3, 5])
    assert np.all(stg[ok] == 0)
    # the autograd wrapper says so
    import torch
    net = gpu.Network(spec)
    p = torch.zeros(spec.n_reactions, dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.warns(RuntimeWarning, match="2 of 20 cells did not reach t_end"):
        Y, E, st = gpu.BurnFn.apply(p, net, bad.Y, bad.rho, bad.T, cfg.t_end)
    assert torch.isfinite(E).all()
    net.close()
    # a step budget smaller than the burn needs
    Yg, Tg, Eg, stg, cntg, gg = _run_gpu(gpu, spec, cells, cfg.t_end, gY, gE, max_steps=5)
    assert np.all(stg == 1) and np.all(gg == 0.0)


def test_adjoint21_full_size_sampled(gpu, oracle):
    """The sensitivity workload as bench.py times it (21/60 network, 65,536
    cells); the oracle's forward sensitivities of a seeded sample of 96
    cells give the reference end states and vector-Jacobian products."""
    import torch
    cfg = synth.config(5)
    spec, cells = cfg.networks[0], cfg.cells[0]
    C = cells.n_cells
    assert C == 65536
    gY, gE = _cot(spec, C, 11)
    net = gpu.Network(spec)
    run = gpu.AdjointRun(net, cells.Y, cells.rho, cells.T, cfg.t_end, RTOL, ATOL)
    Y, T, E, st = run.forward()
    grad = run.backward(gY, gE)
    torch.cuda.synchronize()
    Yg, Tg, stg = Y.cpu().numpy(), T.cpu().numpy(), st.cpu().numpy()
    cntg, gg = run.counters.cpu().numpy(), grad.cpu().numpy()
    net.close()
    assert np.all(stg == 0)
    idx = np.sort(np.random.default_rng(3).choice(C, 96, replace=False))
    sub = cells.subset(idx)
    onet = oracle.OracleNet(spec)
    Yo, To, sto, cnto, S, unc = oracle.sens(onet, sub, cfg.t_end, RTOL, ATOL)

    def tight(i):
        r = oracle.burn(onet, sub.subset(i), cfg.t_end, RTOL * 1e-4, ATOL * 1e-4)
        return r[0], r[1]

    rep = assert_parity((Yg[:, idx], Tg[idx], stg[idx], cntg[:, idx]), (Yo, To, sto, cnto),
                        RTOL, ATOL, tight=tight)
    go = oracle.vjp(onet, S, gY[:, idx], gE[idx])
    same = rep["same_counters"] & (sto == 0)
    scale = np.abs(go).max(axis=0)
    err = np.abs(gg[:, idx] - go).max(axis=0)
    print(f"adjoint full size: sample 96, same schedule {int(same.sum())}, max rel grad err "
          f"{(err / np.maximum(scale, 1e-300)).max():.3e}", flush=True)
    assert same.all()
    assert np.all(err <= GRAD_RTOL * scale + 1e-300)
