"""CPU checks of the adjoint.

* The oracle's FP64 adjoint (forward-mode Jacobians of every reaction
  substep, the transposed diffusion operator, dK/dsigma from its definition)
  against central finite differences of the oracle's own loss, with the k
  decisions frozen by replaying the recorded k-trace (the loss is piecewise
  smooth in the parameters; l does not move for these perturbations).
* The library's hand-written reverse-mode substep (the code the GPU kernel
  instantiates), evaluated on the host in FP64, against fourth-order finite
  differences of the library's forward substep.
"""
import numpy as np
import pytest

from paper_2011_04747_amd import workloads as W


def _make(model, sigma, scal):
    if model == "tp06":
        w = W.adjoint_slab(shape=(9, 7, 5), t_end=6.0, n_sensors=20)
    elif model == "tp06fibro":
        # myocytes and passive fibroblasts (30% of the nodes), stimulated at t = 0
        w = W.sheet_fibrotic_tp06(n=9, dx=0.02, fib_frac=0.3, s1_time=0.0, t_end=6.0)
        w.sensors = np.array([1, 12, 22, 31, 40, 50, 62, 77], np.int32)
    elif model == "tp06types":
        # endocardial, M and epicardial columns of a small transmural sheet
        w = W.sheet_transmural_tp06(n_wall=9, n_height=7, t_end=6.0)
        w.sensors = np.array([1, 12, 22, 31, 40, 50, 62], np.int32)
    else:
        w = W.cable_ms(n_nodes=31, length=0.3, t_end=8.0)
        w.sensors = np.array([3, 10, 20, 29], np.int32)
    w.mesh.sigma = sigma
    p = w.params.copy()
    if model != "ms":
        p[1:6] *= scal[:5, None]
        if model == "tp06fibro" and len(scal) > 5:
            p[7:9] *= scal[5:7, None]        # fibroblast g_f and E_f rows
    else:
        p *= scal[:, None]
    w.params = p
    return w


@pytest.mark.parametrize("model", ["ms", "tp06", "tp06types", "tp06fibro"])
def test_oracle_adjoint_matches_finite_differences(oracle_mod, model):
    rng = np.random.default_rng(1)
    nsc = 7 if model == "tp06fibro" else 5
    w = _make(model, None, np.ones(nsc))
    n = w.mesh.n_nodes
    sig = np.exp(0.1 * rng.standard_normal(n))
    scal = np.ones(nsc)
    w = _make(model, sig, scal)
    o = oracle_mod.Oracle.from_workload(w)
    ns = w.n_steps
    target = rng.uniform(-0.1, 0.1, (ns, len(w.sensors))) + (0.0 if model == "ms" else -80.0)
    kt, _ = o.record_k(ns)
    o.set_target(w.sensors, target)
    o.forward_taped(ns, w.dt)
    gs, gp = o.backward()

    def loss_at(sig2, scal2):
        w2 = _make(model, sig2, scal2)
        o2 = oracle_mod.Oracle.from_workload(w2)
        o2.replay_k(kt)
        o2.set_target(w2.sensors, target)
        return o2.forward_taped(ns, w2.dt)

    for a in rng.choice(n, 4, replace=False):
        eps = 1e-4
        sp, sm = sig.copy(), sig.copy()
        sp[a] *= 1 + eps
        sm[a] *= 1 - eps
        fd = (loss_at(sp, scal) - loss_at(sm, scal)) / (2 * eps * sig[a])
        assert gs[a] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(gs).max())
    if model == "tp06fibro":
        assert gp[6] == 0.0             # the node class is a label
    for b in range(nsc):
        eps = 1e-5
        sp, sm = scal.copy(), scal.copy()
        sp[b] += eps
        sm[b] -= eps
        fd = (loss_at(sig, sp) - loss_at(sig, sm)) / (2 * eps)
        ga = gp[b] if model == "ms" else (gp[b + 1] if b < 5 else gp[b + 2])
        assert ga == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(gp).max())


@pytest.mark.parametrize("model,S,P", [(4, 19, 9), (3, 19, 7), (2, 19, 6), (1, 2, 5), (0, 1, 2)])
@pytest.mark.parametrize("trial", range(6))
def test_library_substep_vjp_matches_finite_differences(model, S, P, trial):
    from paper_2011_04747_amd import mono
    rng = np.random.default_rng(10 + trial)
    y = W.random_state(model, 1, 100 + trial)[:, 0]
    if model in (2, 3, 4):
        y[0] = (-85.0, -60.0, -39.9, -41.0, 10.0, 14.99999)[trial]
        p = np.array(W.TP06_PARAM_DEFAULT) * rng.uniform(0.7, 1.3, 6)
        if model == 3:
            p = np.append(p, (W.CELL_EPI, W.CELL_ENDO, W.CELL_M)[trial % 3])
        if model == 4:
            p = np.append(p, [(W.NODE_MYOCYTE, W.NODE_FIBROBLAST)[trial % 2],
                              0.0216 * rng.uniform(0.7, 1.3), -49.6 * rng.uniform(0.7, 1.3)])
    elif model == 1:
        p = np.array(W.MS_PARAM_DEFAULT)
        y[0] = (0.05, 0.08, 0.3, 0.6, 0.9, 0.95)[trial]      # away from v_gate
    else:
        p = np.array([0.3, -20.0])
    h = 0.02
    lam = rng.standard_normal(S)
    l_in, gp = mono.model_vjp_host(model, y, p, h, lam)

    def f(yy, pp):
        return lam @ mono.model_substep_host(model, yy, pp, h)

    def d4(fun, x, a, e):
        xp, xm, xp2, xm2 = x.copy(), x.copy(), x.copy(), x.copy()
        xp[a] += e; xm[a] -= e; xp2[a] += 2 * e; xm2[a] -= 2 * e
        return (8 * (fun(xp) - fun(xm)) - (fun(xp2) - fun(xm2))) / (12 * e)

    for a in range(S):
        e = 1e-3 * max(abs(y[a]), 1e-4)
        fd = d4(lambda x: f(x, p), y, a, e)
        assert l_in[a] == pytest.approx(fd, rel=2e-6, abs=1e-7 * np.abs(l_in).max()), a
    if model in (3, 4):
        assert gp[6] == 0.0          # the cell type / node class is a label
    for b in [q for q in range(P) if not (model in (3, 4) and q == 6)]:
        e = 1e-3 * max(abs(p[b]), 1e-4)
        fd = d4(lambda x: f(y, x), p, b, e)
        assert gp[b] == pytest.approx(fd, rel=2e-6, abs=1e-7 * max(np.abs(gp).max(), 1e-12)), b
