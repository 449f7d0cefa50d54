"""GPU adjoint (FP32) against the FP64 oracle adjoint and against FP64 central
differences of the oracle forward run; autograd wrapper.

The loss is L = 1/2 |rho_T - target|^2, so grad_final = rho_T - target.  The
GPU gradient differs from the oracle's by the FP32 rounding of both the
forward replay and the reverse solves (about 1e-6 relative); the bound used
is 1e-4 relative to each quantity's largest magnitude.
"""
from __future__ import annotations

import copy

import numpy as np
import pytest

import oracle as O
from paper_2110_13368_amd import binding as vb
from paper_2110_13368_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _case(seed, shape, n_sub=2, bc="mixed", n_cells=40, h=(20.0, 20.0, 20.0), dt=0.01):
    rng = np.random.default_rng(seed)
    spec = W.make_sim(rng, shape, h, n_sub, dtype="f32", bc=bc, n_cells=n_cells, cell_layout="uniform", dt=dt)
    if n_cells > 2:
        spec.cells.pos[1] = spec.cells.pos[0]  # two cells in one voxel
        spec.cells.pos[2] = spec.cells.pos[0]
    target = rng.uniform(0, 40, size=spec.field_shape)
    return spec, target


def _oracle_grads(spec, target, mode, n_steps):
    sim = O.from_spec(spec, decay_mode=mode)
    sim.step(n_steps)
    r = sim.get_field() - target
    sim.set_field(spec.rho0.astype(np.float64))
    return sim.adjoint(n_steps, r), r


def _gpu_grads(specs, finals, mode, n_steps, ckpt, x_lanes=0):
    """GPU gradients; x_lanes None tunes the launch configuration first, as the
    benchmark does (tuning overwrites the field, which is then set again)."""
    decay = vb.VL_DECAY_ONCE if mode == O.DECAY_ONCE else vb.VL_DECAY_THIRDS
    ctx = vb.Context(specs, decay_split=decay, device="cuda:0")
    try:
        if x_lanes is None:
            ctx.tune(None)
            for k, s in enumerate(specs):
                ctx.set_field(k, s.rho0)
            print(f"tuned: x lanes {ctx.get_option(vb.VL_OPT_X_LANES)}, "
                  f"lines per wave {ctx.get_option(vb.VL_OPT_X_LANE_LINES)}", flush=True)
        else:
            ctx.set_option(vb.VL_OPT_X_LANES, x_lanes)
        before = [ctx.get_field(k).copy() for k in range(len(specs))]
        g = ctx.adjoint(n_steps, ckpt, [f.astype(np.float32) for f in finals])
        out = [{k: (v.double().cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)) for k, v in d.items()}
               for d in g]
        after = [ctx.get_field(k) for k in range(len(specs))]
        for a, b in zip(before, after):
            assert np.array_equal(a, b), "field not restored after the adjoint"
        return out
    finally:
        ctx.close()


def _close(got, want, what, tol=TOL):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if want.size == 0:
        return
    scale = float(np.max(np.abs(want)))
    err = float(np.max(np.abs(got - want)))
    print(f"{what}: max |err| {err:.3e}, scale {scale:.3e}", flush=True)
    assert err <= tol * max(scale, 1e-30), f"{what}: {err:.3e} > {tol} x {scale:.3e}"


def _compare(g, o, what):
    _close(g["rho0"], o["rho0"], what + " grad_rho0")
    _close(g["D"], o["D"], what + " dD")
    _close(g["lambda"], o["lambda"], what + " dlambda")
    _close(g["S"], o["S"], what + " dS")
    _close(g["U"], o["U"], what + " dU")


@pytest.mark.parametrize("mode", [O.DECAY_ONCE, O.DECAY_THIRDS])
@pytest.mark.parametrize("shape,bc", [((23, 17, 11), "mixed"), ((9, 30, 14), "dirichlet"),
                                      ((16, 16, 16), "neumann")])
def test_adjoint_matches_oracle(mode, shape, bc):
    spec, target = _case(11 + shape[0], shape, bc=bc)
    n_steps = 7
    o, r = _oracle_grads(spec, target, mode, n_steps)
    g = _gpu_grads([spec], [r], mode, n_steps, ckpt=3)[0]
    _compare(g, o, f"{shape} {bc} mode {mode}")


@pytest.mark.parametrize("mode", [O.DECAY_ONCE, O.DECAY_THIRDS])
@pytest.mark.parametrize("shape,x_lanes", [((130, 13, 9), 1), ((100, 11, 7), 2), ((70, 6, 5), 2)])
def test_adjoint_with_x_lanes_forward(mode, shape, x_lanes):
    # forward steps and replays use the lanes-along-the-line x solve
    spec, target = _case(123, shape, bc="mixed", n_cells=30)
    o, r = _oracle_grads(spec, target, mode, 6)
    g = _gpu_grads([spec], [r], mode, 6, ckpt=4, x_lanes=x_lanes)[0]
    _compare(g, o, f"x lanes {x_lanes} {shape} mode {mode}")


@pytest.mark.parametrize("mode", [O.DECAY_ONCE, O.DECAY_THIRDS])
def test_adjoint_long_lines_and_degenerate_axes(mode):
    # lines of 1, 2, 3 voxels and lines in the larger capacity classes
    cases = [((1, 2, 3), 0), ((130, 3, 2), 6), ((2, 201, 1), 6), ((5, 4, 257), 10),
             ((3, 401, 2), 6), ((513, 2, 1), 6)]
    for shape, nc in cases:
        spec, target = _case(500 + sum(shape), shape, bc="mixed", n_cells=nc)
        o, r = _oracle_grads(spec, target, mode, 4)
        g = _gpu_grads([spec], [r], mode, 4, ckpt=2)[0]
        _compare(g, o, f"{shape} mode {mode}")


@pytest.mark.parametrize("mode", [O.DECAY_ONCE, O.DECAY_THIRDS])
@pytest.mark.parametrize("shape,h,x_lanes", [((150, 40, 1), (10.0, 15.0, 10.0), 1),
                                             ((31, 70, 1), (20.0, 20.0, 20.0), 0),
                                             ((24, 18, 13), (8.0, 20.0, 35.0), 0),
                                             ((140, 9, 6), (12.0, 5.0, 30.0), 1)])
def test_adjoint_two_dimensional_and_unequal_edges(mode, shape, h, x_lanes):
    # grids one voxel thick (2-D) and voxels with unequal edges
    spec, target = _case(321 + sum(shape), shape, bc="mixed", n_cells=30, h=h)
    if shape[2] == 1:
        spec.bc_kind[:, 4:] = 0
        spec.bc_value[:, 4:] = 0.0
    o, r = _oracle_grads(spec, target, mode, 6)
    g = _gpu_grads([spec], [r], mode, 6, ckpt=4, x_lanes=x_lanes)[0]
    _compare(g, o, f"{shape} h={h} mode {mode}")


def test_adjoint_batched_ragged():
    specs, targets = [], []
    for k, shape in enumerate([(20, 13, 9), (33, 8, 17), (7, 7, 40)]):
        s, t = _case(900 + k, shape, n_sub=1 + k % 2, bc="mixed", n_cells=25 + 10 * k)
        specs.append(s)
        targets.append(t)
    n_steps = 5
    res = [_oracle_grads(s, t, O.DECAY_ONCE, n_steps) for s, t in zip(specs, targets)]
    g = _gpu_grads(specs, [r for _, r in res], O.DECAY_ONCE, n_steps, ckpt=2)
    for k, (o, _) in enumerate(res):
        _compare(g[k], o, f"sim {k}")


def test_adjoint_checkpoint_spacing_is_exact():
    # the replay is deterministic, so the spacing of checkpoints cannot change
    # a single bit of the result
    spec, target = _case(77, (19, 12, 10))
    _, r = _oracle_grads(spec, target, O.DECAY_ONCE, 6)
    ref = _gpu_grads([spec], [r], O.DECAY_ONCE, 6, ckpt=1)[0]
    for ckpt in (2, 4, 6, 50):
        g = _gpu_grads([spec], [r], O.DECAY_ONCE, 6, ckpt=ckpt)[0]
        for key in ref:
            assert np.array_equal(g[key], ref[key]), (ckpt, key)


@pytest.mark.parametrize("x_lanes", [1, 2])
def test_adjoint_x_lanes_reverse_batch_and_checkpoints(x_lanes):
    """Reverse x solves with the lanes along the line next to split ones: a
    batch of x-lines of 150, 100, 70 and 40 voxels (lanes for 129+, or 65+
    with setting 2; split below), against the oracle, and bitwise equal for
    every checkpoint spacing."""
    specs, targets = [], []
    for k, shape in enumerate([(150, 5, 6), (100, 7, 4), (70, 6, 5), (40, 9, 3)]):
        s, t = _case(950 + k, shape, n_sub=1 + k % 2, bc="mixed", n_cells=20 + 5 * k)
        specs.append(s)
        targets.append(t)
    n_steps = 4
    res = [_oracle_grads(s, t, O.DECAY_ONCE, n_steps) for s, t in zip(specs, targets)]
    finals = [r for _, r in res]
    ref = _gpu_grads(specs, finals, O.DECAY_ONCE, n_steps, ckpt=1, x_lanes=x_lanes)
    for k, (o, _) in enumerate(res):
        _compare(ref[k], o, f"x lanes {x_lanes} sim {k}")
    for ckpt in (2, 3, 4):
        g = _gpu_grads(specs, finals, O.DECAY_ONCE, n_steps, ckpt=ckpt, x_lanes=x_lanes)
        for k in range(len(specs)):
            for key in ref[k]:
                assert np.array_equal(g[k][key], ref[k][key]), (x_lanes, ckpt, k, key)


def test_adjoint_zero_steps_and_out_of_domain_cell():
    spec, target = _case(31, (12, 11, 10))
    spec.cells.pos[5] = np.array(spec.lo) - 5.0
    g = _gpu_grads([spec], [target], O.DECAY_ONCE, 0, ckpt=1)[0]
    assert np.array_equal(g["rho0"], target.astype(np.float32).astype(np.float64))
    assert np.all(g["D"] == 0) and np.all(g["lambda"] == 0)
    assert np.all(g["S"] == 0) and np.all(g["U"] == 0)
    o, r = _oracle_grads(spec, target, O.DECAY_ONCE, 3)
    g = _gpu_grads([spec], [r], O.DECAY_ONCE, 3, ckpt=2)[0]
    assert np.all(g["S"][5] == 0) and np.all(g["U"][5] == 0)
    _compare(g, o, "out-of-domain cell")


def _oracle_loss(spec, target, mode, n_steps, **over):
    sp = copy.deepcopy(spec)
    for k, v in over.items():
        if k in ("S", "U"):
            setattr(sp.cells, k, v)
        else:
            setattr(sp, k, v)
    sim = O.from_spec(sp, decay_mode=mode)
    sim.step(n_steps)
    d = sim.get_field() - target
    return 0.5 * float(np.sum(d * d))


@pytest.mark.parametrize("mode", [O.DECAY_ONCE, O.DECAY_THIRDS])
def test_adjoint_sixteen_parameters_vs_fp64_central_differences(mode):
    """The differentiation workload (Gaussian cell ball, zero-flux faces, two
    substrates) at 40^3 voxels and 1280 cells, 20 steps with checkpoints every
    5: D and lambda of both substrates and S, U of six cells, against FP64
    central differences of the oracle's forward run."""
    wl = W.differentiation(scale=0.4)
    spec = wl.sims[0]
    rng = np.random.default_rng(4242)
    target = spec.rho0.astype(np.float64) + rng.normal(0, 1.0, size=spec.field_shape)
    n_steps = 20
    o, r = _oracle_grads(spec, target, mode, n_steps)
    g = _gpu_grads([spec], [r], mode, n_steps, ckpt=5)[0]
    vox = O.from_spec(spec).cell_voxels()
    inside = [i for i in range(spec.cells.n) if vox[i] >= 0][:6]
    checks = []

    # The loss is about 1e7, so a central difference with a tiny step is lost
    # in rounding; Richardson extrapolation of central differences with
    # relative steps 2e-2 and 1e-2 leaves an O(h^4) truncation error.
    def central(name, idx, base, hstep):
        p, m = base.copy(), base.copy()
        p[idx] += hstep
        m[idx] -= hstep
        return (_oracle_loss(spec, target, mode, n_steps, **{name: p})
                - _oracle_loss(spec, target, mode, n_steps, **{name: m})) / (2 * hstep)

    def fd(name, idx, base):
        h = 2e-2 * abs(base[idx])
        return (4.0 * central(name, idx, base, h / 2) - central(name, idx, base, h)) / 3.0

    for s in range(2):
        checks.append(("D", s, g["D"][s], fd("D", s, spec.D), o["D"][s]))
        checks.append(("lambda", s, g["lambda"][s], fd("lam", s, spec.lam), o["lambda"][s]))
    for j, i in enumerate(inside):
        s = j % 2
        checks.append(("S", (i, s), g["S"][i, s], fd("S", (i, s), spec.cells.S), o["S"][i, s]))
        checks.append(("U", (i, s), g["U"][i, s], fd("U", (i, s), spec.cells.U), o["U"][i, s]))
    assert len(checks) == 16
    for name, idx, got, want, orc in checks:
        print(f"{name}{idx}: gpu {got:.8e} fd {want:.8e} oracle {orc:.8e}", flush=True)
        assert abs(got - want) <= TOL * abs(want), (name, idx, got, want)
        assert abs(got - orc) <= TOL * abs(orc), (name, idx, got, orc)


def test_autograd_function_and_parameter_update():
    import torch

    from paper_2110_13368_amd.autograd import LODStepFn, flat_params

    spec, target = _case(61, (14, 10, 12), bc="mixed", n_cells=30)
    n_steps = 4
    ctx = vb.Context([spec], device="cuda:0")
    try:
        D, lam, S, U = flat_params(ctx)
        D2 = (D * 1.3).requires_grad_()
        lam2 = (lam * 0.7).requires_grad_()
        S2 = (S * 1.1).requires_grad_()
        U2 = (U * 0.9).requires_grad_()
        rho0 = ctx.to_field_layout([spec.rho0]).requires_grad_()
        out = LODStepFn.apply(rho0, D2, lam2, S2, U2, ctx, n_steps, 3)
        rho_t = ctx.from_field_layout(out, 0)
        tgt = torch.as_tensor(target, dtype=torch.float32, device="cuda:0")
        loss = 0.5 * ((rho_t - tgt) ** 2).sum()
        loss.backward()

        sp = copy.deepcopy(spec)
        sp.D, sp.lam = D2.detach().numpy(), lam2.detach().numpy()
        sp.cells.S = S2.detach().numpy().reshape(-1, spec.n_sub)
        sp.cells.U = U2.detach().numpy().reshape(-1, spec.n_sub)
        o, _ = _oracle_grads(sp, target, O.DECAY_ONCE, n_steps)
        fwd = O.from_spec(sp)
        fwd.step(n_steps)
        _close(rho_t.detach().double().cpu().numpy(), fwd.get_field(), "forward with updated parameters", 1e-5)
        _close(ctx.from_field_layout(rho0.grad, 0).double().cpu().numpy(), o["rho0"], "autograd grad_rho0")
        _close(D2.grad.numpy(), o["D"], "autograd dD")
        _close(lam2.grad.numpy(), o["lambda"], "autograd dlambda")
        _close(S2.grad.cpu().numpy().reshape(-1, spec.n_sub), o["S"], "autograd dS")
        _close(U2.grad.cpu().numpy().reshape(-1, spec.n_sub), o["U"], "autograd dU")
    finally:
        ctx.close()


# --------------------------------------------------------------------------
# The differentiation workload at its stated size: 100^3 x 2, 2e4 cells in a
# Gaussian ball, 200 FP32 steps with a checkpoint every 20.  The loss is
# L = 1/2 |rho_T - target|^2 with the target a forward run whose D, lambda, S
# and U are multiplied by exp(0.1 N(0, 1)) (seeded).  Sixteen parameters: D and
# lambda of both substrates and S or U of twelve seeded-random in-domain cells,
# against FP64 central differences of the oracle with h = 1e-6 |p|.  The loss
# is about 1e6, so L(p + h) - L(p - h) formed from two rounded losses would
# lose the difference; it is formed from the fields instead, as
#   1/2 sum (rho+ - rho-) (rho+ + rho- - 2 target),
# which equals it exactly in real arithmetic.

DIFF_STEPS, DIFF_CKPT, DIFF_H = 200, 20, 1e-6


@pytest.fixture(scope="module")
def differentiation_case():
    wl = W.differentiation()
    spec = wl.sims[0]
    assert wl.steps == DIFF_STEPS and spec.shape == (100, 100, 100) and spec.cells.n == 20000
    rng = np.random.default_rng(W.SEED_BASE + 4004)
    pert = copy.deepcopy(spec)
    pert.D = spec.D * np.exp(0.1 * rng.normal(size=spec.D.shape))
    pert.lam = spec.lam * np.exp(0.1 * rng.normal(size=spec.lam.shape))
    pert.cells.S = spec.cells.S * np.exp(0.1 * rng.normal(size=spec.cells.S.shape))
    pert.cells.U = spec.cells.U * np.exp(0.1 * rng.normal(size=spec.cells.U.shape))
    tsim = O.from_spec(pert)
    tsim.step(DIFF_STEPS)
    target = tsim.get_field()
    tsim.close()
    o, r = _oracle_grads(spec, target, O.DECAY_ONCE, DIFF_STEPS)
    g = _gpu_grads([spec], [r], O.DECAY_ONCE, DIFF_STEPS, ckpt=DIFF_CKPT, x_lanes=None)[0]
    vox = O.from_spec(spec).cell_voxels()
    inside = np.flatnonzero(vox >= 0)
    cells = rng.choice(inside, size=12, replace=False)
    params = [("D", s) for s in range(2)] + [("lam", s) for s in range(2)]
    params += [("S" if j % 2 == 0 else "U", (int(i), int(rng.integers(0, 2)))) for j, i in enumerate(cells)]
    return spec, target, o, g, params


def _field_after(spec, name, idx, value):
    sp = copy.deepcopy(spec)
    arr = (sp.cells.S if name == "S" else sp.cells.U if name == "U" else sp.D if name == "D" else sp.lam).copy()
    arr[idx] = value
    if name in ("S", "U"):
        setattr(sp.cells, name, arr)
    else:
        setattr(sp, name, arr)
    sim = O.from_spec(sp)
    sim.step(DIFF_STEPS)
    f = sim.get_field()
    sim.close()
    return f


def _central(spec, target, name, idx):
    base = {"S": spec.cells.S, "U": spec.cells.U, "D": spec.D, "lam": spec.lam}[name]
    p = float(base[idx])
    h = DIFF_H * abs(p)
    fp = _field_after(spec, name, idx, p + h)
    fm = _field_after(spec, name, idx, p - h)
    return 0.5 * float(np.sum((fp - fm) * (fp + fm - 2.0 * target))) / (2.0 * h)


def test_differentiation_workload_gpu_adjoint_matches_oracle_adjoint(differentiation_case):
    spec, _, o, g, _ = differentiation_case
    _compare(g, o, "100^3x2, 200 steps, checkpoints every 20")


@pytest.mark.parametrize("part", range(4))
def test_differentiation_workload_sixteen_parameters_vs_fd(differentiation_case, part):
    spec, target, o, g, params = differentiation_case
    assert len(params) == 16
    key = {"D": "D", "lam": "lambda", "S": "S", "U": "U"}
    for name, idx in params[4 * part:4 * part + 4]:
        fd = _central(spec, target, name, idx)
        got = float(g[key[name]][idx])
        orc = float(o[key[name]][idx])
        print(f"{name}{idx}: gpu {got:.8e}  oracle adjoint {orc:.8e}  fd(h=1e-6|p|) {fd:.8e}  "
              f"rel gpu {abs(got - fd) / abs(fd):.2e}  rel oracle {abs(orc - fd) / abs(fd):.2e}", flush=True)
        # The oracle's adjoint is the exact FP64 transpose.  What separates it
        # from the central difference is the difference's own error: at
        # h = 1e-6 |p| on this size the two FP64 forward runs' rounding no
        # longer cancels (spatially correlated noise of ~1e-12 per voxel over
        # 2e6 voxels), e.g. 3.5e-5 relative on D of substrate 1, while a
        # difference at h = 1e-4 |p| agrees with the adjoint to 9e-8.  So both
        # adjoints are held to the configuration's 1e-4 against it; the GPU
        # and oracle adjoints are compared array by array in the test above.
        assert abs(orc - fd) <= TOL * abs(fd), (name, idx, orc, fd)
        assert abs(got - fd) <= TOL * abs(fd), (name, idx, got, fd)


def _fewer_cells(cells, n):
    c = copy.deepcopy(cells)
    c.pos, c.V, c.S, c.U, c.rho_star = c.pos[:n], c.V[:n], c.S[:n], c.U[:n], c.rho_star[:n]
    return c


def test_adjoint_after_reupload_with_fewer_cells():
    """Per-cell gradients are laid out by the cells uploaded now: in a batch of
    two, simulation 0 is re-uploaded with fewer cells; both simulations' dS and
    dU (and the rest) must match the oracle's adjoint for the cells in place."""
    s0, t0 = _case(1201, (18, 14, 11), n_cells=40)
    s1, t1 = _case(1202, (15, 16, 12), n_cells=30)
    n_steps = 5
    ctx = vb.Context([s0, s1], device="cuda:0")
    try:
        fewer = _fewer_cells(s0.cells, 17)
        ctx.upload_cells(0, fewer)
        assert ctx.n_cells(0) == 17 and ctx.n_cells(1) == 30
        s0b = copy.copy(s0)
        s0b.cells = fewer
        o0, r0 = _oracle_grads(s0b, t0, O.DECAY_ONCE, n_steps)
        o1, r1 = _oracle_grads(s1, t1, O.DECAY_ONCE, n_steps)
        g = ctx.adjoint(n_steps, 2, [r0.astype(np.float32), r1.astype(np.float32)])
        g = [{k: (v.double().cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)) for k, v in d.items()} for d in g]
        assert g[0]["S"].shape == (17, 2) and g[1]["S"].shape == (30, 2)
        _compare(g[0], o0, "re-uploaded sim 0")
        _compare(g[1], o1, "sim 1 after sim 0's re-upload")
    finally:
        ctx.close()


def test_autograd_keeps_cells_moved_on_the_device():
    """After a device upload of moved cells, autograd's forward pass with new
    S, U re-uploads the moved positions, not the spec's original ones."""
    import torch

    from paper_2110_13368_amd.autograd import LODStepFn, flat_params

    spec, target = _case(1301, (16, 12, 10), bc="mixed", n_cells=25)
    n_steps = 4
    ctx = vb.Context([spec], device="cuda:0")
    try:
        moved = copy.deepcopy(spec.cells)
        moved.pos = moved.pos + np.array([spec.h[0], -0.5 * spec.h[1], 0.0])
        moved.pos[:, 0] = np.minimum(moved.pos[:, 0], spec.lo[0] + spec.shape[0] * spec.h[0] - 1.0)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
        ctx.upload_cells_device(0, dev(moved.pos), dev(moved.V), dev(moved.S), dev(moved.U), dev(moved.rho_star))
        D, lam, S, U = flat_params(ctx)
        S2, U2 = (S * 1.2).requires_grad_(), (U * 0.8).requires_grad_()
        rho0 = ctx.to_field_layout([spec.rho0]).requires_grad_()
        out = LODStepFn.apply(rho0, D, lam, S2, U2, ctx, n_steps, 2)
        sp = copy.deepcopy(spec)
        sp.cells = moved
        sp.cells.S = S2.detach().numpy().reshape(-1, spec.n_sub)
        sp.cells.U = U2.detach().numpy().reshape(-1, spec.n_sub)
        fwd = O.from_spec(sp)
        fwd.step(n_steps)
        _close(ctx.from_field_layout(out, 0).detach().double().cpu().numpy(), fwd.get_field(),
               "forward with moved cells and new rates", 1e-5)
        loss = 0.5 * ((ctx.from_field_layout(out, 0) - torch.as_tensor(target, dtype=torch.float32,
                                                                       device="cuda:0")) ** 2).sum()
        loss.backward()
        o, _ = _oracle_grads(sp, target, O.DECAY_ONCE, n_steps)
        _close(S2.grad.cpu().numpy().reshape(-1, spec.n_sub), o["S"], "dS with moved cells")
        _close(U2.grad.cpu().numpy().reshape(-1, spec.n_sub), o["U"], "dU with moved cells")
    finally:
        ctx.close()


def test_uploads_without_adjoint_tables():
    """VL_OPT_ADJOINT_TABLES 0: uploads skip the per-cell tables only the
    adjoint reads.  The forward fields are bitwise those of uploads that write
    them; vl_adjoint refuses (VL_E_STATE) until the cells are uploaded again
    with the tables, and then matches the oracle's adjoint."""
    spec, target = _case(1301, (17, 13, 10), n_cells=40)
    n_steps = 4
    fields = []
    for tables in (1, 0):
        ctx = vb.Context([spec], device="cuda:0")
        try:
            ctx.set_option(vb.VL_OPT_ADJOINT_TABLES, tables)
            ctx.upload_cells(0, spec.cells)
            ctx.step(n_steps)
            ctx.sync()
            fields.append(ctx.get_field(0).copy())
            if tables == 0:
                ctx.set_field(0, spec.rho0)
                with pytest.raises(vb.VoxlodError) as e:
                    ctx.adjoint(n_steps, 2, [np.zeros(spec.field_shape, np.float32)])
                assert e.value.code == vb.VL_E_STATE
                ctx.set_option(vb.VL_OPT_ADJOINT_TABLES, 1)
                ctx.upload_cells(0, spec.cells)
                o, r = _oracle_grads(spec, target, O.DECAY_ONCE, n_steps)
                g = ctx.adjoint(n_steps, 2, [r.astype(np.float32)])
                g = {k: (v.double().cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)) for k, v in g[0].items()}
                _compare(g, o, "after re-upload with the tables")
        finally:
            ctx.close()
    assert np.array_equal(fields[0], fields[1])


def test_adjoint_with_z_sources_while_storing():
    """The adjoint's checkpointed forward and segment replays with the z
    tiles applying the cell sources while they store (forced on; these small
    fields leave it off by default) give bitwise the gradients of the pass
    after the stores, and the oracle's."""
    spec, target = _case(1401, (19, 15, 70), n_cells=300)
    n_steps = 6
    o, r = _oracle_grads(spec, target, O.DECAY_ONCE, n_steps)
    got = []
    for storing in (1, 0):
        ctx = vb.Context([spec], device="cuda:0")
        try:
            ctx.set_option(vb.VL_OPT_FUSE_SOURCES, 1)
            ctx.set_option(vb.VL_OPT_Z_SOURCES_STORING, storing)
            g = ctx.adjoint(n_steps, 2, [r.astype(np.float32)])
            got.append({k: (v.double().cpu().numpy() if hasattr(v, "cpu") else np.asarray(v))
                        for k, v in g[0].items()})
        finally:
            ctx.close()
    for k in got[0]:
        assert np.array_equal(got[0][k], got[1][k]), f"{k}: while storing vs after the stores"
    _compare(got[0], o, "z sources while storing")
