"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (set in the tests below):
  * basis, ranks, occupations: bit-exact;
  * H psi: relative 2-norm error <= 1e-13 (rounding of a sum of <= M^3 terms);
  * amplitudes after RK4: ||psi_gpu - psi_cpu||_2 <= 1e-10;
  * observables: relative error <= 1e-9.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle, dense, derived, evolve, states

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_00050_amd as fh  # noqa: E402


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _pair(M, sectors, omega, Lam, V):
    return Oracle(M, M, omega, Lam, V, sectors), fh.Model(M, omega, Lam, V), fh.Basis(M, sectors)


# ----------------------------------------------------------------- basis ---
BASIS_CASES = [(1, 7), (2, 9), (3, 11), (4, 12), (5, 8), (5, 14), (6, 13), (7, 9), (8, 8), (9, 6), (10, 6)]


@pytest.mark.parametrize("M,N", BASIS_CASES)
def test_basis_bitexact(M, N):
    sectors = [(N, p) for p in range(M)] + [(0, 0), (1, 1 % M)]
    orc = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), sectors)
    b = fh.Basis(M, sectors)
    assert b.dims == orc.dims
    assert b.offsets[:-1] == orc.offsets
    occ = b.occupations().cpu().numpy()
    want = orc.all_occupations()
    assert np.array_equal(occ, want)
    for s in range(len(sectors)):
        o = torch.from_numpy(orc.occupations(s)).cuda()
        idx = b.rank(s, o).cpu().numpy()
        assert np.array_equal(idx, np.arange(orc.dims[s]))
        back = b.unrank(s, torch.arange(orc.dims[s], dtype=torch.int64, device="cuda")).cpu().numpy()
        assert np.array_equal(back, orc.occupations(s))
    # vectors of another sector rank to -1
    if M > 1:
        o = torch.from_numpy(orc.occupations(0)).cuda()
        assert np.all(b.rank(1, o).cpu().numpy() == -1)


# ---------------------------------------------------------------- H psi ---
def _model(kind, M, seed):
    if kind == "contact":
        return W.omega_quadratic(M), W.V_contact(M)
    if kind == "longrange":
        return W.omega_quadratic(M), W.V_longrange(M)
    if kind == "sym":
        return np.random.default_rng(seed).uniform(-1, 1, M), W.V_random_symmetric(M, seed)
    return np.random.default_rng(seed).uniform(-1, 1, M), W.V_random(M, seed)


HPSI_CASES = [
    (1, [(n, 0) for n in range(0, 12)], "sym"),
    (2, [(9, 0), (9, 1), (3, 1)], "nonsym"),
    (3, [(12, p) for p in range(3)], "sym"),
    (4, [(11, p) for p in range(4)] + [(2, 0)], "nonsym"),
    (5, [(8, 2)], "contact"),
    (5, [(12, p) for p in range(5)], "longrange"),
    (6, [(10, p) for p in range(6)], "sym"),
    (6, [(n, p) for n in range(0, 8) for p in range(6)], "contact"),
    (7, [(8, 3), (7, 1)], "nonsym"),
    (8, [(8, 0), (8, 5)], "longrange"),
    (8, [(7, p) for p in range(8)], "sym"),
    (9, [(6, 2), (6, 0)], "nonsym"),
    (10, [(6, p) for p in range(10)], "contact"),
    (10, [(5, 3), (6, 7)], "sym"),
]


@pytest.mark.parametrize("M,sectors,kind", HPSI_CASES, ids=[f"M{c[0]}-{c[2]}-{len(c[1])}sec" for c in HPSI_CASES])
def test_apply_h_vs_oracle(M, sectors, kind):
    omega, V = _model(kind, M, 100 + M)
    orc, model, b = _pair(M, sectors, omega, 0.37, V)
    x = W.random_psi(orc.total, 7)
    want = orc.apply_h(x)
    got = fh.apply_h(model, b, torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(got, want) <= 1e-13


@pytest.mark.parametrize("M,nrhs", [(6, 2), (6, 4), (6, 8), (6, 16), (8, 8), (10, 16)])
def test_apply_h_multi_rhs(M, nrhs):
    Nmax = {6: 9, 8: 6, 10: 4}[M]
    sectors = [(Nmax, p) for p in range(M)] + [(Nmax - 1, 1)]
    omega, V = _model("longrange", M, 3)
    orc, model, b = _pair(M, sectors, omega, 0.21, V)
    X = W.random_psi(orc.total, 17, nrhs=nrhs)
    got = fh.apply_h(model, b, torch.from_numpy(X).cuda()).cpu().numpy()
    for q in range(nrhs):
        # every column is summed in the single-rhs order: bitwise equal
        single = fh.apply_h(model, b, torch.from_numpy(np.ascontiguousarray(X[:, q])).cuda()).cpu().numpy()
        assert np.array_equal(got[:, q], single)
        assert _rel(got[:, q], orc.apply_h(np.ascontiguousarray(X[:, q]))) <= 1e-13


# -------------------------------------------------------------- moments ---
@pytest.mark.parametrize("M,Nmax", [(1, 9), (2, 8), (3, 8), (5, 6), (6, 6), (8, 4), (10, 3)])
def test_moments_vs_oracle(M, Nmax):
    sectors = W.all_sectors(M, Nmax)
    orc = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), sectors)
    b = fh.Basis(M, sectors)
    x = W.random_psi(orc.total, 5)
    n2, a, Mm, A = fh.moments(b, torch.from_numpy(x).cuda())
    wn2, wa, wM, wA = orc.moments(x)
    scale = wn2
    assert abs(n2 - wn2) <= 1e-12 * scale
    assert np.abs(a - wa).max() <= 1e-12 * scale
    assert np.abs(Mm - wM).max() <= 1e-12 * scale * Nmax
    assert np.abs(A - wA).max() <= 1e-12 * scale * Nmax


def test_moments_missing_partner_sectors():
    """Terms whose image lies outside the retained sectors count as zero."""
    M = 4
    sectors = [(6, 1), (5, 0), (6, 3), (4, 2)]
    orc = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), sectors)
    b = fh.Basis(M, sectors)
    x = W.random_psi(orc.total, 8)
    got = fh.moments(b, torch.from_numpy(x).cuda())
    want = orc.moments(x)
    for g, w in zip(got, want):
        assert np.allclose(g, w, rtol=0, atol=1e-12 * want[0])


def test_derive_matches_oracle_on_gpu_moments():
    M = 4
    alpha = W.coherent_amplitudes(9, M, 2.5)
    sectors = W.all_sectors(M, 16)
    orc = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), sectors)
    b = fh.Basis(M, sectors)
    psi = fh.init_coherent(b, alpha)
    got = fh.derive(M, *fh.moments(b, psi))
    want = derived.observe(orc, states.coherent_state(orc, alpha))
    for k in ("n_tot", "lambda_p", "vminus"):
        assert abs(got[k] - want[k]) <= 1e-9 * max(1.0, abs(want[k]))
    assert abs(got["Q"] - want["Q"]) <= 1e-9


# ---------------------------------------------------------- initial states ---
def test_initial_states_vs_oracle():
    M = 5
    sectors = W.all_sectors(M, 9)
    orc = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), sectors)
    b = fh.Basis(M, sectors)
    al = np.stack([W.coherent_amplitudes(s, M, 2.0) for s in (1, 2)])
    got = fh.init_coherent(b, al).cpu().numpy()
    for q in range(2):
        assert _rel(got[:, q], states.coherent_state(orc, al[q])) <= 1e-13
    z = W.coherent_amplitudes(3, M, 4.0)
    b6 = fh.Basis(M, [(6, p) for p in range(M)])
    o6 = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), [(6, p) for p in range(M)])
    assert _rel(fh.init_fieldnumber(b6, z).cpu().numpy(), states.fieldnumber_state(o6, z)) <= 1e-13
    n = [2, 0, 1, 3, 0]
    bn = fh.Basis(M, [(6, W.momentum(n, M))])
    on = Oracle(M, M, np.zeros(M), 0.0, np.zeros((M,) * 4), [(6, W.momentum(n, M))])
    assert np.array_equal(fh.init_number(bn, n).cpu().numpy(), states.number_state(on, n))


# ------------------------------------------------------------------ RK4 ---
def _oracle_run(orc, psi0, dt, nsteps, every):
    return evolve.rk4(orc, psi0, dt, nsteps, every=every, observe=lambda s, t, p: orc.moments(p))


def _check_records(M, res, recs, rhs=0):
    """Relative 1e-9 on every observable.  Q = (n_tot - sum|<a>|^2)/n_tot and
    V_- are differences of O(n_tot) terms, so each also gets an absolute floor
    of 1e-12 (n_tot rounding, ~1e-16 n_tot, amplified by the cancellation)."""
    assert len(res.records) == len(recs)
    for r, (n2, a, Mm, A) in zip(res.records[:, rhs], recs):
        g = fh.derive(M, *fh.unpack_moments(M, r))
        o = derived.derive(n2, a, Mm, A)
        for k in ("norm2", "n_tot", "lambda_p"):
            assert abs(g[k] - o[k]) <= 1e-9 * max(abs(o[k]), 1e-300), k
        floor = 1e-12 * max(1.0, o["n_tot"])
        assert abs(g["Q"] - o["Q"]) <= 1e-9 * abs(o["Q"]) + floor
        if np.isfinite(o["vminus"]):
            assert abs(g["vminus"] - o["vminus"]) <= 1e-9 * abs(o["vminus"]) + floor
        assert np.all(np.abs(g["vminus_mode"] - o["vminus_mode"]) <= 1e-9 * np.abs(o["vminus_mode"]) + floor)
        for k in ("a", "M", "A"):
            assert np.abs(g[k] - o[k]).max() <= 1e-9 * np.abs(o[k]).max() + floor, k
        np.testing.assert_allclose(g["n_modes"], np.real(np.diag(o["M"])), rtol=1e-9, atol=floor)


def test_rk4_tiny_number_state_full_run():
    w = W.tiny_number()
    orc, model, b = _pair(w.M, w.sectors, w.omega, w.Lambda, w.V)
    psi = fh.init_number(b, w.init_params)
    res = fh.evolve_rk4(model, b, psi, w.dt, w.nsteps, every=w.every)
    ref, recs = _oracle_run(orc, states.number_state(orc, w.init_params), w.dt, w.nsteps, w.every)
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(w.M, res, recs)


@pytest.mark.parametrize("flags", [0, fh.FH_PER_SECTOR, fh.FH_GRAPH, fh.FH_TIMING])
def test_rk4_coherent_multisector(flags):
    M, Lam = 4, 0.3
    alpha = W.coherent_amplitudes(13, M, 2.0)
    sectors = W.all_sectors(M, 12)
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    psi = fh.init_coherent(b, alpha)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        res = fh.evolve_rk4(model, b, psi, 2e-3, 150, every=50, flags=flags)
    stream.synchronize()
    ref, recs = _oracle_run(orc, states.coherent_state(orc, alpha), 2e-3, 150, 50)
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(M, res, recs)
    if flags & fh.FH_TIMING:
        assert res.stage_launches == 4 * 150 and res.stage_ms > 0


@pytest.mark.parametrize("c2,flags", [(0.5, 0), (1.0, 0), (0.5, fh.FH_GRAPH), (0.5, fh.FH_PER_SECTOR)])
def test_taylor2_vs_oracle(c2, flags):
    """The paper's second-order step (Eq. Q_int) on the GPU against the oracle's."""
    M, Lam, dt, nsteps, every = 4, 0.3, 1e-3, 120, 40
    alpha = W.coherent_amplitudes(17, M, 2.0)
    sectors = W.all_sectors(M, 12)
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    psi = fh.init_coherent(b, alpha)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        res = fh.evolve_taylor2(model, b, psi, dt, nsteps, c2=c2, every=every, flags=flags)
    stream.synchronize()
    ref, recs = evolve.taylor2(orc, states.coherent_state(orc, alpha), dt, nsteps, c2=c2, every=every,
                               observe=lambda s, t, p: orc.moments(p))
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(M, res, recs)


def test_batched_equals_per_sector_bitwise():
    M = 5
    alpha = W.coherent_amplitudes(2, M, 3.0)
    sectors = W.all_sectors(M, 14)
    model = fh.Model(M, W.omega_quadratic(M), 0.05, W.V_contact(M))
    b = fh.Basis(M, sectors)
    p1 = fh.init_coherent(b, alpha)
    p2 = p1.clone()
    fh.evolve_rk4(model, b, p1, 1e-3, 40)
    fh.evolve_rk4(model, b, p2, 1e-3, 40, flags=fh.FH_PER_SECTOR)
    assert torch.equal(p1, p2)


@pytest.mark.parametrize("blocks_per_cu,xcd_order",
                         [(0, 1), (1, 0), (2, 1), (0, 2), (3, 2), (0, 3), (1, 3), (2, 3)])
def test_schedule_does_not_change_results(blocks_per_cu, xcd_order):
    """Tile order, persistent grid size and XCD mapping only change which
    workgroup computes a row, never the row's arithmetic (one and four
    columns; a fused RK4 step too)."""
    M = 6
    sectors = W.all_sectors(M, 16)
    model = fh.Model(M, W.omega_quadratic(M), 0.05, W.V_longrange(M))
    b = fh.Basis(M, sectors)
    x = torch.from_numpy(W.random_psi(b.total, 3)).cuda()
    x4 = torch.from_numpy(W.random_psi(b.total, 4, 4)).cuda()
    ref, ref4 = fh.apply_h(model, b, x), fh.apply_h(model, b, x4)
    y = x.clone()
    fh.evolve_rk4(model, b, y, 1e-3, 2)
    b.set_launch(blocks_per_cu, xcd_order)
    for order, prefix in ((1, 3), (0, 0), (1, 2), (0, 4), (1, 5)):
        b.set_tile_order(order, prefix)
        assert torch.equal(fh.apply_h(model, b, x), ref)
        assert torch.equal(fh.apply_h(model, b, x4), ref4)
    z = x.clone()
    fh.evolve_rk4(model, b, z, 1e-3, 2)
    assert torch.equal(z, y)


def test_rk4_fieldnumber_multi_rhs():
    M, N, nrhs = 5, 7, 4
    n = np.array([3, 1, 0, 2, 1])
    z = W.phase_draws(n, range(50, 50 + nrhs))
    sectors = [(N, p) for p in range(M)]
    omega, V = W.omega_linear(M), W.V_contact(M)
    orc, model, b = _pair(M, sectors, omega, 0.1, V)
    psi = fh.init_fieldnumber(b, z)
    res = fh.evolve_rk4(model, b, psi, 5e-3, 60, every=30)
    got = psi.cpu().numpy()
    for q in range(nrhs):
        ref, recs = _oracle_run(orc, states.fieldnumber_state(orc, z[q]), 5e-3, 60, 30)
        assert np.linalg.norm(got[:, q] - ref) <= 1e-10
        _check_records(M, res, recs, rhs=q)


# ----------------------------------------------------- large sector, sampled ---
def test_large_sector_sampled():
    """The benchmark's sector (M=8, N=48, P=0): dimension, sampled ranks and
    sampled rows of H psi against the oracle, in the benchmark's launch setup."""
    w = W.large_sector()
    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    b = fh.Basis(w.M, w.sectors)
    assert b.total == orc.total == 25_366_335
    rng = np.random.default_rng(4)
    rows = np.sort(np.concatenate([rng.choice(b.total, 3000, replace=False), [0, 1, b.total - 1]]))
    occ_all = orc.occupations(0)
    occ = occ_all[rows]
    got_occ = b.unrank(0, torch.from_numpy(rows).cuda()).cpu().numpy()
    assert np.array_equal(got_occ, occ)
    assert np.array_equal(b.rank(0, torch.from_numpy(np.ascontiguousarray(occ)).cuda()).cpu().numpy(), rows)
    x = W.random_psi(b.total, 21)
    got = fh.apply_h(model, b, torch.from_numpy(x).cuda()).cpu().numpy()[rows]
    want = orc.apply_h_rows(x, rows)
    assert _rel(got, want) <= 1e-13
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


# -------------------------------------------------------------- adjoint ---
def test_adjoint_vs_oracle():
    M, Lam, dt, nsteps = 3, 0.35, 5e-3, 30
    sectors = W.all_sectors(M, 9)
    omega = W.omega_quadratic(M)
    V = W.V_longrange(M) + 0.3 * W.V_contact(M)
    alpha = W.coherent_amplitudes(31, M, 1.5)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    psi0o = states.coherent_state(orc, alpha)
    for obj, mk in ((fh.FH_J_Q, evolve.objective_Q), (fh.FH_J_PO, evolve.objective_PO),
                    (fh.FH_J_NMODE, lambda o: evolve.objective_mode_occupation(o, 1))):
        ref = evolve.adjoint(orc, psi0o, dt, nsteps, mk(orc))
        psi0 = fh.init_coherent(b, alpha)
        res = fh.adjoint_rk4(model, b, psi0, dt, nsteps, 7, obj, mode=1)
        # recomputing the stage inputs instead of keeping them changes no bit
        res2 = fh.adjoint_rk4(model, b, psi0, dt, nsteps, 7, obj, mode=1, keep_stage_inputs=False)
        assert np.array_equal(res["lambda0"].cpu().numpy(), res2["lambda0"].cpu().numpy())
        assert res["dLambda"][0] == res2["dLambda"][0] and np.array_equal(res["dV"], res2["dV"])
        # one segment (every state and stage input kept from the forward sweep) changes no bit
        res3 = fh.adjoint_rk4(model, b, psi0, dt, nsteps, nsteps, obj, mode=1)
        assert np.array_equal(res["lambda0"].cpu().numpy(), res3["lambda0"].cpu().numpy())
        assert res["dLambda"][0] == res3["dLambda"][0] and np.array_equal(res["dV"], res3["dV"])
        assert abs(res["J"][0] - ref["J"]) <= 1e-10
        assert abs(res["dLambda"][0] - ref["dLambda"]) <= 1e-9 * max(1, abs(ref["dLambda"]))
        # only momentum-conserving entries are parameters of the model; the
        # others are reported as exactly zero
        cons = W.V_contact(M) != 0
        assert np.abs(res["dV"][0][cons] - ref["dV"][cons]).max() <= 1e-9 * max(1, np.abs(ref["dV"]).max())
        assert np.all(res["dV"][0][~cons] == 0)
        lam0 = res["lambda0"].cpu().numpy()
        assert _rel(lam0, ref["g0"]) <= 1e-10
        dre, dim = fh.coherent_vjp(b, alpha, res["lambda0"])
        wre, wim = evolve.coherent_alpha_gradient(orc, alpha, psi0o, ref["g0"])
        assert np.abs(dre[0] - wre).max() <= 1e-9 * max(1, np.abs(wre).max())
        assert np.abs(dim[0] - wim).max() <= 1e-9 * max(1, np.abs(wim).max())


def test_qevolve_gradcheck():
    """torch.autograd binding: its backward equals central differences of its
    forward for Re alpha, Im alpha, Lambda and every momentum-conserving V
    entry (the non-conserving ones are not parameters of the model)."""
    from paper_2111_00050_amd.autograd import EvolveSpec, QEvolve

    M = 3
    b = fh.Basis(M, W.all_sectors(M, 8))
    spec = EvolveSpec(b, W.omega_quadratic(M), 1e-2, 40, ckpt_every=9, objective=fh.FH_J_Q)
    cons = torch.as_tensor(np.flatnonzero(W.V_contact(M).ravel() != 0))
    V0 = (W.V_longrange(M) + 0.3 * W.V_contact(M)).ravel()
    a = W.coherent_amplitudes(31, M, 1.2)
    f64 = dict(dtype=torch.float64, requires_grad=True)
    are, aim = torch.tensor(a.real, **f64), torch.tensor(a.imag, **f64)
    lam = torch.tensor(0.6, **f64)
    vc = torch.tensor(V0[cons.numpy()], **f64)

    def J(are, aim, lam, vc):
        V = torch.zeros(M ** 4, dtype=torch.float64).index_put((cons,), vc).reshape(M, M, M, M)
        return QEvolve.apply(are, aim, lam, V, spec)

    assert float(J(are, aim, lam, vc).detach()) > 1e-3  # a nontrivial Q
    assert torch.autograd.gradcheck(J, (are, aim, lam, vc), eps=1e-6, atol=1e-8, rtol=1e-5)


def test_autotune_changes_no_bit(tmp_path):
    """The autotuner only picks a launch schedule: H psi is bitwise unchanged,
    the pick is one of the candidates and a second basis reads it back from
    the cache file."""
    M = 6
    sectors = [(12, p) for p in range(M)]
    omega, V = _model("longrange", M, 5)
    orc, model, b = _pair(M, sectors, omega, 0.2, V)
    x = torch.from_numpy(W.random_psi(orc.total, 9)).cuda()
    before = fh.apply_h(model, b, x).cpu().numpy()
    cache = tmp_path / "tune.txt"
    cfg, ms = fh.autotune(model, b, x, cache_path=cache)
    assert ms > 0
    assert cfg["blocks_per_cu"] in (0, 1, 2, 3) and cfg["xcd_order"] in (0, 1, 2, 3)
    assert cfg["prefix_modes"] in (0, 2, 3) and cfg["tile_order"] == (1 if cfg["prefix_modes"] else 0)
    assert np.array_equal(fh.apply_h(model, b, x).cpu().numpy(), before)
    assert _rel(before, orc.apply_h(x.cpu().numpy())) <= 1e-13
    b2 = fh.Basis(M, sectors)
    cfg2, ms2 = fh.autotune(model, b2, x, cache_path=cache)
    assert cfg2 == cfg and ms2 == pytest.approx(ms, rel=1e-5)
    assert np.array_equal(fh.apply_h(model, b2, x).cpu().numpy(), before)


@pytest.mark.parametrize("keep", [True, False])
def test_adjoint_two_rhs_matches_single(keep):
    """Two coherent states adjointed together give, column by column, what
    each gives alone (the multi-rhs stage kernel sums each column in the
    single-rhs order).  With kept stage inputs the correlators run on
    contiguous copies of each column; without, at M = 4 (four pairs per
    launch) two columns leave too few free scratch vectors for the copies and
    the correlators gather every other 16 bytes of the interleaved vector."""
    M, Lam, dt, nsteps = 4, 0.3, 5e-3, 12
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    b = fh.Basis(M, W.all_sectors(M, 8))
    model = fh.Model(M, omega, Lam, V)
    al = np.stack([W.coherent_amplitudes(s, M, 1.3) for s in (61, 62)])
    both = fh.adjoint_rk4(model, b, fh.init_coherent(b, al), dt, nsteps, 5, fh.FH_J_Q, keep_stage_inputs=keep)
    lam_both = both["lambda0"].cpu().numpy()
    for q in range(2):
        one = fh.adjoint_rk4(model, b, fh.init_coherent(b, al[q]), dt, nsteps, 5, fh.FH_J_Q, keep_stage_inputs=keep)
        assert abs(both["J"][q] - one["J"][0]) <= 1e-14
        assert abs(both["dLambda"][q] - one["dLambda"][0]) <= 1e-12 * max(1.0, abs(one["dLambda"][0]))
        assert np.abs(both["dV"][q] - one["dV"][0]).max() <= 1e-12 * max(1.0, np.abs(one["dV"][0]).max())
        assert _rel(lam_both[:, q], one["lambda0"].cpu().numpy()) <= 1e-13


# ------------------------------------------------------- classical field ---
@pytest.mark.parametrize("M,kind", [(1, "sym"), (3, "nonsym"), (5, "longrange"), (8, "sym"), (10, "contact")])
def test_classical_vs_oracle(M, kind):
    from oracle import classical

    omega, V = _model(kind, M, 40 + M)
    Lam, dt, nsteps, every = 0.3, 1e-3, 300, 100
    a0 = np.stack([W.coherent_amplitudes(s, M, 2.0) for s in range(70, 77)])
    model = fh.Model(M, omega, Lam, V)
    aT, traj = fh.classical_rk4(model, a0, dt, nsteps, every)
    wT, wtraj = classical.rk4(omega, Lam, V, a0, dt, nsteps, every)
    assert traj.shape == wtraj.shape
    assert np.abs(traj.cpu().numpy() - wtraj).max() <= 1e-11 * np.abs(wtraj).max()
    assert np.abs(aT.cpu().numpy() - wT).max() <= 1e-11 * np.abs(wT).max()


def test_classical_equals_quantum_mean_without_interaction():
    """Lambda = 0: <a_p>(t) of the evolved coherent state equals the classical
    trajectory from the same amplitudes.  Exactly so for the flows; the two RK4
    discretisations differ by their truncation error (each quantum term gets
    R(+i E' dt) R(-i E dt) per step instead of R(-i w_p dt)), below 1e-12 at
    this step size for the occupations that carry the weight."""
    M, dt, nsteps = 4, 1e-3, 200
    omega = W.omega_quadratic(M)
    alpha = W.coherent_amplitudes(5, M, 1.5)
    model = fh.Model(M, omega, 0.0, W.V_contact(M))
    b = fh.Basis(M, W.all_sectors(M, 22))
    psi = fh.init_coherent(b, alpha)
    res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=nsteps)
    n2, a_q, _, _ = fh.unpack_moments(M, res.records[-1, 0])
    aT, _ = fh.classical_rk4(model, alpha, dt, nsteps)
    # the truncated coherent state keeps 1 - n2 ~ 1e-9 of its norm outside the sectors
    assert np.abs(a_q / n2 - aT.cpu().numpy()[0]).max() <= 1e-8


# ---------------------------------------------------- forward-mode tangent ---
def test_tangent_dlambda_matches_adjoint():
    """Forward-mode d/dLambda of the RK4 map gives the same dJ/dLambda as the
    oracle's discrete adjoint (pinned by P12) and as the GPU adjoint."""
    M, Lam, dt, nsteps = 3, 0.35, 5e-3, 30
    sectors = W.all_sectors(M, 9)
    omega = W.omega_quadratic(M)
    V = W.V_longrange(M) + 0.3 * W.V_contact(M)
    alpha = W.coherent_amplitudes(31, M, 1.5)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    psi0o = states.coherent_state(orc, alpha)
    for obj, mk in ((fh.FH_J_Q, evolve.objective_Q), (fh.FH_J_PO, evolve.objective_PO),
                    (fh.FH_J_NMODE, lambda o: evolve.objective_mode_occupation(o, 1))):
        ref = evolve.adjoint(orc, psi0o, dt, nsteps, mk(orc))
        psi0 = fh.init_coherent(b, alpha)
        tan = fh.tangent_rk4(model, b, psi0, dt, nsteps, obj, mode=1)
        assert abs(tan["J"][0] - ref["J"]) <= 1e-10
        assert abs(tan["dLambda"][0] - ref["dLambda"]) <= 1e-9 * max(1, abs(ref["dLambda"]))
        adj = fh.adjoint_rk4(model, b, psi0, dt, nsteps, 7, obj, mode=1)
        assert abs(tan["dLambda"][0] - adj["dLambda"][0]) <= 1e-10 * max(1, abs(adj["dLambda"][0]))


def test_tangent_two_rhs():
    M, Lam, dt, nsteps = 4, 0.3, 5e-3, 12
    b = fh.Basis(M, W.all_sectors(M, 8))
    model = fh.Model(M, W.omega_quadratic(M), Lam, W.V_longrange(M))
    al = np.stack([W.coherent_amplitudes(s, M, 1.3) for s in (61, 62)])
    both = fh.tangent_rk4(model, b, fh.init_coherent(b, al), dt, nsteps, fh.FH_J_Q)
    for q in range(2):
        one = fh.tangent_rk4(model, b, fh.init_coherent(b, al[q]), dt, nsteps, fh.FH_J_Q)
        assert abs(both["J"][q] - one["J"][0]) <= 1e-14
        assert abs(both["dLambda"][q] - one["dLambda"][0]) <= 1e-12 * max(1.0, abs(one["dLambda"][0]))


# ---------------------------------------------------- Chebyshev propagator ---
def test_chebyshev_vs_oracle_and_exponential():
    """Large steps (|E| dt far past RK4's limit): equal to the oracle's series
    and to the dense exponential."""
    w = W.tiny_number()
    orc, model, b = _pair(w.M, w.sectors, w.omega, w.Lambda, w.V)
    H = dense.dense_h(orc)
    E = np.linalg.eigvalsh(H)
    emin, emax = E.min() - 0.5, E.max() + 0.5
    dt, n = 0.7, 5
    psi = fh.init_number(b, w.init_params)
    res = fh.evolve_chebyshev(model, b, psi, dt, n, emin, emax, every=1)
    psi0 = states.number_state(orc, w.init_params)
    ref, recs = evolve.chebyshev(orc, psi0, dt, n, emin, emax, every=1, observe=lambda s, t, p: orc.moments(p))
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-12
    assert np.linalg.norm(psi.cpu().numpy() - dense.expm_evolve(H, psi0, n * dt)) <= 1e-11
    _check_records(w.M, res, recs)


@pytest.mark.parametrize("flags", [0, fh.FH_PER_SECTOR])
def test_chebyshev_multisector_vs_rk4(flags):
    """Coherent state over many sectors: a few Chebyshev steps agree with many
    small RK4 steps to the RK4 error; bounds from the power iteration."""
    M, Lam = 4, 0.3
    alpha = W.coherent_amplitudes(13, M, 2.0)
    sectors = W.all_sectors(M, 12)
    orc, model, b = _pair(M, sectors, W.omega_quadratic(M), Lam, W.V_longrange(M))
    psi_c = fh.init_coherent(b, alpha)
    fh.evolve_chebyshev(model, b, psi_c, 0.1, 3, flags=flags)
    psi_r = fh.init_coherent(b, alpha)
    fh.evolve_rk4(model, b, psi_r, 1e-4, 3000)
    assert _rel(psi_c.cpu().numpy(), psi_r.cpu().numpy()) <= 1e-9


def test_spectral_radius_power_iteration():
    w = W.tiny_number()
    orc, model, b = _pair(w.M, w.sectors, w.omega, w.Lambda, w.V)
    rho = np.abs(np.linalg.eigvalsh(dense.dense_h(orc))).max()
    est = fh.spectral_radius(model, b, iters=300)
    assert 0.95 * rho <= est <= rho * (1 + 1e-12)


def test_chebyshev_rejects_a_too_small_interval():
    w = W.tiny_number()
    orc, model, b = _pair(w.M, w.sectors, w.omega, w.Lambda, w.V)
    rho = np.abs(np.linalg.eigvalsh(dense.dense_h(orc))).max()
    psi = fh.init_number(b, w.init_params)
    with pytest.raises(fh.FockError):
        fh.evolve_chebyshev(model, b, psi, 2.0, 20, -0.2 * rho, 0.2 * rho)


# ------------------------------------------------------------ edge cases ---
def test_empty_and_single_state_sectors():
    """Sectors with no states (N = 0, P != 0) and with one state sit in the
    basis without effect: evolution and moments match the oracle."""
    M = 4
    sectors = [(0, 1), (0, 0), (1, 3), (5, 2), (4, 0), (3, 1)]
    omega, V = _model("sym", M, 5)
    orc, model, b = _pair(M, sectors, omega, 0.4, V)
    assert b.dims[0] == 0 and b.dims[1] == 1
    x = W.random_psi(orc.total, 21)
    assert _rel(fh.apply_h(model, b, torch.from_numpy(x).cuda()).cpu().numpy(), orc.apply_h(x)) <= 1e-13
    psi = torch.from_numpy(x).cuda()
    res = fh.evolve_rk4(model, b, psi, 1e-2, 30, every=10)
    ref, recs = _oracle_run(orc, x, 1e-2, 30, 10)
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(M, res, recs)


def test_vacuum_only_basis():
    """The one-state basis {|0>}: H|0> = 0 and every moment but the norm vanishes."""
    M = 3
    model, b = fh.Model(M, W.omega_quadratic(M), 0.5, W.V_contact(M)), fh.Basis(M, [(0, 0)])
    psi = torch.tensor([0.6 - 0.8j], dtype=torch.complex128, device="cuda")
    assert torch.count_nonzero(fh.apply_h(model, b, psi)) == 0
    res = fh.evolve_rk4(model, b, psi, 0.1, 5, every=5)
    n2, a, Mij, Akl = fh.unpack_moments(M, res.records[-1, 0])
    assert abs(n2 - 1.0) <= 1e-15 and not a.any() and not Mij.any() and not Akl.any()


def test_classical_edge_arguments():
    M = 3
    model = fh.Model(M, W.omega_quadratic(M), 0.2, W.V_contact(M))
    a0 = W.coherent_amplitudes(3, M, 1.0)
    aT, traj = fh.classical_rk4(model, a0, 1e-2, 0, every=1)  # zero steps: only the initial record
    assert traj.shape == (1, 1, M) and np.array_equal(traj.cpu().numpy()[0, 0], a0)
    assert np.array_equal(aT.cpu().numpy()[0], a0)
    aT2, none = fh.classical_rk4(model, a0, 1e-2, 10)
    assert none is None and aT2.shape == (1, M)


def test_error_returns_are_exceptions():
    """Invalid calls come back as FockError with the library's message and
    launch nothing."""
    M = 3
    model, b = fh.Model(M, W.omega_quadratic(M), 0.2, W.V_contact(M)), fh.Basis(M, W.all_sectors(M, 4))
    x = torch.from_numpy(W.random_psi(b.total, 1, nrhs=3)).cuda()
    with pytest.raises(fh.FockError, match="nrhs"):
        fh.apply_h(model, b, x)
    y = torch.from_numpy(W.random_psi(b.total, 1)).cuda()
    with pytest.raises(fh.FockError, match="alias"):
        fh.apply_h(model, b, y, out=y)
    other = fh.Model(M + 1, W.omega_quadratic(M + 1), 0.2, W.V_contact(M + 1))
    with pytest.raises(fh.FockError, match="disagree"):
        fh.apply_h(other, b, y)
    with pytest.raises(fh.FockError, match="emin < emax"):
        fh.evolve_chebyshev(model, b, y, 0.1, 1, 1.0, -1.0)


# ---------------------------------------------- exact momentum (Sec. IV.A) ---
def _exact_oracle(w, sectors_exact):
    pmod = max(N for N, _ in sectors_exact) * (w.M - 1) + 1
    return Oracle(w.M, pmod, w.omega, w.Lambda, w.V, sectors_exact)


def _rows_of(b, orc):
    """GPU basis row of every oracle (exact-sector) state, matched by occupations."""
    occ = b.occupations().cpu().numpy()
    row = {o.tobytes(): r for r, o in enumerate(occ)}
    return np.array([row[o.tobytes()] for o in orc.all_occupations()], np.int64)


@pytest.mark.parametrize("inter", ["longrange", "contact+", "contact-"])
def test_paper_number_state_exact_momentum(inter):
    """|0, 2r, 2r, r, 0> (r = 2) with the paper's exactly conserving
    interactions: the periodic sector holding it evolves, on the GPU, exactly as
    the oracle's exact sector (Sigma j n_j = 18) and every other state stays 0."""
    w = W.paper_problem("number", inter, 2)
    N, P = w.sectors[0]
    orc = _exact_oracle(w, [(N, w.meta["P_exact"])])
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    rows = _rows_of(b, orc)
    assert b.total > orc.total
    psi = fh.init_number(b, w.init_params)
    dt, nsteps, every = 2e-3, 400, 100
    res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=every)
    ref, recs = _oracle_run(orc, states.number_state(orc, w.init_params), dt, nsteps, every)
    got = psi.cpu().numpy()
    assert np.linalg.norm(got[rows] - ref) <= 1e-10
    rest = np.ones(b.total, bool)
    rest[rows] = False
    assert np.all(got[rest] == 0)
    _check_records(w.M, res, recs)


@pytest.mark.parametrize("init,inter", [("coherent", "longrange"), ("coherent", "contact-"),
                                        ("fieldnumber", "longrange")])
def test_paper_superpositions_exact_momentum(init, inter):
    """Coherent and field-number states of the paper's test problems (r = 1):
    all periodic sectors together equal all exact sectors; amplitudes and
    observables on the GPU match the oracle run in the exact basis, and so do
    the breaktimes Q = 0.15 (coherent states) and 1 - lambda_p/n_tot = 0.1
    extracted from both.  The run lasts to t = 3.6, past every compared crossing
    (the latest, the long-range field-number PO crossing, lies near t = 2.9)."""
    w = W.paper_problem(init, inter, 1)
    z = w.init_params[0]
    if init == "coherent":
        Nmax = 10
        sectors = W.all_sectors(w.M, Nmax)
        exact = [(N, P) for N in range(Nmax + 1) for P in range(N * (w.M - 1) + 1)]
    else:
        sectors = w.sectors
        N = sectors[0][0]
        exact = [(N, P) for P in range(N * (w.M - 1) + 1)]
    orc = _exact_oracle(w, exact)
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, sectors)
    rows = _rows_of(b, orc)
    assert sorted(rows.tolist()) == list(range(b.total))
    if init == "coherent":
        psi, ref0 = fh.init_coherent(b, z), states.coherent_state(orc, z)
    else:
        psi, ref0 = fh.init_fieldnumber(b, z), states.fieldnumber_state(orc, z)
    assert _rel(psi.cpu().numpy()[rows], ref0) <= 1e-13
    dt, nsteps, every = 1e-2, 360, 5
    res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=every)
    ref, recs = evolve.rk4(orc, ref0, dt, nsteps, every=every, observe=lambda s, t, p: orc.moments(p))
    assert np.linalg.norm(psi.cpu().numpy()[rows] - ref) <= 1e-10
    _check_records(w.M, res, recs)
    ser = fh.observable_series(w.M, res, dt)
    t = np.arange(len(recs)) * every * dt
    want = [derived.derive(*r) for r in recs]
    # Q of a field-number state is 1 at every time (fixed N), so its crossing
    # is the first sample and says nothing; compare the PO crossing there.
    keys = (("Q", fh.BREAK_Q), ("po_deficit", fh.BREAK_PO)) if init == "coherent" else (("po_deficit", fh.BREAK_PO),)
    if init == "fieldnumber":
        assert all(abs(d["Q"] - 1.0) <= 1e-12 for d in want)
    for key, level in keys:
        ref_t = fh.first_crossing(t, np.array([d[key] for d in want]), level)
        got_t = fh.first_crossing(ser["t"], ser[key], level)
        assert 0.0 < ref_t < nsteps * dt, (key, ref_t)
        assert abs(got_t - ref_t) <= 1e-8, (key, got_t, ref_t)


def test_breaktime_sweep_runner_agrees_with_rk4():
    """The sweep runner (Chebyshev records every 0.02) and a plain RK4 run
    (dt = 1e-3, records every 0.02) give the same Q breaktime of the paper's
    contact problem at r = 1 (Sec. IV.C), up to RK4's truncation."""
    import os
    import sys

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads"))
    import breaktime_sweep as S

    out = S.run("coherent-contact+", 1, 0.02, 1.0, None, 1.1, classical=True, t_ref=0.5)
    assert out["states"] == 8568 and out["sectors"] == 70
    # at t = 0 the quantum occupations are |z_k|^2 up to the 0.999 truncation
    assert out["classical"]["dev_at_0"] < 5e-3 and out["classical"]["dev_max"] > out["classical"]["dev_at_0"]
    w = W.paper_problem("coherent", "contact+", 1)
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, W.all_sectors(w.M, S.poisson_nmax(5.0)))
    psi = fh.init_coherent(b, w.init_params[0])
    res = fh.evolve_rk4(model, b, psi, 1e-3, 1000, every=20)
    bt = fh.breaktimes(fh.observable_series(w.M, res, 1e-3))
    assert 0.5 < out["t_Q"] < 0.7
    for k in ("t_Q", "t_PO", "t_sqz"):
        assert abs(out[k] - bt[k]) <= 1e-6, k


# ------------------------------------------------------ full-size samples ---
def _sample_rows(orc, rng, n):
    """Random rows plus the first and last row of every fifth sector."""
    edges = []
    for s in range(0, len(orc.sectors), 5):
        if orc.dims[s]:
            edges += [orc.offsets[s], orc.offsets[s] + orc.dims[s] - 1]
    return np.unique(np.concatenate([rng.choice(orc.total, n, replace=False), edges])).astype(np.int64)


def test_batched_coherent_full_size_sampled():
    """The batched workload at full size (M=6, 541 sectors, 927,048,304 states):
    one persistent H psi launch over all sectors, sampled rows against the oracle."""
    w = W.batched_coherent()
    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    assert b.total == orc.total == 927_048_304
    rows = _sample_rows(orc, np.random.default_rng(8), 3000)
    x = W.periodic_psi(b.total, 3)
    xd = torch.from_numpy(x).cuda()
    out = fh.apply_h(model, b, xd)
    del xd
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    del out
    want = orc.apply_h_rows(x, rows)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_fieldnumber_sixteen_rhs_full_size_sampled():
    """The 16-draw workload at full size (M=10, N=30, all P: 211,915,132 states
    x 16 right-hand sides): column q holds e^{i phi_q} x0, so its sampled rows of
    H psi must be e^{i phi_q} times the oracle's rows for x0; a column mix-up
    would show the wrong phase."""
    w = W.fieldnumber_draws()
    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, w.sectors)
    assert b.total == orc.total == 211_915_132
    rows = _sample_rows(orc, np.random.default_rng(9), 2000)
    x0 = W.periodic_psi(b.total, 5)
    ph = np.exp(1j * np.linspace(0.3, 5.9, 16))
    X = torch.from_numpy(x0).cuda()[:, None] * torch.from_numpy(ph).cuda()[None, :]
    out = fh.apply_h(model, b, X.contiguous())
    del X
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    del out
    want = orc.apply_h_rows(x0, rows)
    scale = np.abs(want).max()
    for q in range(16):
        assert np.abs(got[:, q] - ph[q] * want).max() <= 1e-13 * scale, q


# ------------------------------------------------- adjoint at full size ---
def _terminal_J(model, b, psi0, dt, nsteps, obj, mode):
    psi = psi0.clone()
    res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=nsteps)
    d = fh.derive(b.M, *fh.unpack_moments(b.M, res.records[-1, 0]))
    if obj == fh.FH_J_Q:
        return d["Q"]
    if obj == fh.FH_J_PO:
        return d["po_deficit"]
    return float(np.real(d["M"][mode, mode]))


@pytest.mark.parametrize("which", ["number", "coherent"])
def test_adjoint_full_size_central_differences(which):
    """The adjoint workloads at full size (M=6, long range, Lambda = 0.03: a number
    state N=30, 54,132 states, 3000 steps, checkpoints every 100, J = <n_0>; a
    coherent state of mean 20, 55,525,372 states, 100 steps, checkpoints every
    10, J = Q): dJ/dLambda, one dJ/dV entry and (coherent) dJ/dRe alpha_0 and
    dJ/dIm alpha_1 against central differences of GPU forward runs."""
    if which == "number":
        w, nsteps, ck, obj, mode = W.adjoint_number(30), 3000, 100, fh.FH_J_NMODE, 0
    else:
        w, nsteps, ck, obj, mode = W.adjoint_coherent(20.0), 100, 10, fh.FH_J_Q, 0
    b = fh.Basis(w.M, w.sectors)

    def init(alpha=None):
        if which == "number":
            return fh.init_number(b, w.init_params)
        return fh.init_coherent(b, w.init_params if alpha is None else alpha)

    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    res = fh.adjoint_rk4(model, b, init(), w.dt, nsteps, ck, obj, mode)
    J0 = _terminal_J(model, b, init(), w.dt, nsteps, obj, mode)
    assert abs(res["J"][0] - J0) <= 1e-12 * max(1.0, abs(J0))

    def cd(fn, h):
        return (fn(h) - fn(-h)) / (2 * h)

    def close(a, want):
        assert abs(a - want) <= 1e-7 * max(1.0, abs(want)), (a, want)

    h = 1e-6
    close(res["dLambda"][0], cd(lambda e: _terminal_J(fh.Model(w.M, w.omega, w.Lambda + e, w.V), b, init(),
                                                      w.dt, nsteps, obj, mode), h))
    # one momentum-conserving entry of V (1 + 2 = 0 + 3 mod 6)
    idx = (1, 2, 0, 3)

    def jv(e):
        V = w.V.copy()
        V[idx] += e
        return _terminal_J(fh.Model(w.M, w.omega, w.Lambda, V), b, init(), w.dt, nsteps, obj, mode)

    close(res["dV"][0][idx], cd(jv, 1e-5))
    if which == "coherent":
        dre, dim = fh.coherent_vjp(b, w.init_params, res["lambda0"])
        a0 = np.array(w.init_params, dtype=np.complex128).reshape(w.M)

        def ja(k, unit):
            def f(e):
                a = a0.copy()
                a[k] += unit * e
                return _terminal_J(model, b, init(a), w.dt, nsteps, obj, mode)
            return f

        close(dre[0][0], cd(ja(0, 1.0), h))
        close(dim[0][1], cd(ja(1, 1j), h))


def test_paper_coherent_full_size_sampled_exact_sectors():
    """The paper's long-range coherent problem at r = 16 (n_tot = 80; Poisson
    weight >= 0.999 keeps N <= 109: 146,803,272 states in 550 periodic sectors):
    one H psi launch over the periodic basis against the oracle's exact sectors
    (Sigma j n_j fixed) on sampled rows.  The vector is a function of the
    occupation vector, so both bases hold the same state; rows are matched by
    occupations through the GPU rank entry point."""
    import os
    import sys

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads"))
    import breaktime_sweep as S

    w = W.paper_problem("coherent", "longrange", 16)
    Nmax = S.poisson_nmax(80.0)
    assert Nmax == 109
    b = fh.Basis(w.M, W.all_sectors(w.M, Nmax))
    assert b.total == 146_803_272
    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    x = W.occupation_psi(b.occupations().cpu().numpy(), 11)
    out = fh.apply_h(model, b, torch.from_numpy(x).cuda())
    del x
    exact = [(40, 80), (80, 161), (100, 200), (109, 218), (109, 300), (109, 0), (109, 1), (109, 436), (1, 3)]
    orc = Oracle(w.M, Nmax * (w.M - 1) + 1, w.omega, w.Lambda, w.V, exact)
    xo = W.occupation_psi(orc.all_occupations(), 11)
    rng = np.random.default_rng(12)
    for s, (N, P) in enumerate(exact):
        loc = np.unique(np.concatenate([rng.choice(orc.dims[s], min(400, orc.dims[s]), replace=False),
                                        [0, orc.dims[s] - 1]]))
        occ = np.ascontiguousarray(orc.occupations(s)[loc])
        ps = N * w.M + P % w.M  # periodic sector (N, P mod M) in all_sectors order
        grow = b.rank(ps, torch.from_numpy(occ).cuda()).cpu().numpy()
        assert np.all(grow >= 0)
        got = out[torch.from_numpy(grow + b.offsets[ps]).cuda()].cpu().numpy()
        want = orc.apply_h_rows(xo, loc + orc.offsets[s])
        assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max()), (N, P)


def test_largest_sector_below_the_limit_sampled():
    """M=8, N=68, P=0: 248,104,707 states, 3.97 GB per vector, the largest M=8
    sector under the 2^28-state limit, where the one-column kernel's 32-bit
    byte offsets come closest to 2^32: sampled rows of H psi (incl. the last
    rows) against the oracle."""
    M, N = 8, 68
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    orc = Oracle(M, M, omega, 0.02, V, [(N, 0)])
    b = fh.Basis(M, [(N, 0)])
    assert b.total == orc.total == 248_104_707
    model = fh.Model(M, omega, 0.02, V)
    x = W.periodic_psi(b.total, 13)
    out = fh.apply_h(model, b, torch.from_numpy(x).cuda())
    rng = np.random.default_rng(14)
    rows = np.unique(np.concatenate([rng.choice(b.total, 3000, replace=False),
                                     np.arange(b.total - 300, b.total), np.arange(300)])).astype(np.int64)
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    want = orc.apply_h_rows(x, rows)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_m10_stages_with_separate_update():
    """M = 10: RK4 and the second-order step against the oracle; 16 columns
    (where a stage is an H y pass plus a separate update pass) bitwise equal to
    single columns (fused epilogue); the adjoint's dJ/dLambda against the
    oracle's adjoint."""
    M, Lam, dt = 10, 0.2, 4e-3
    sectors = [(5, p) for p in range(M)] + [(4, 3)]
    omega, V = W.omega_linear(M), W.V_random_symmetric(M, 21)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    al = np.stack([W.coherent_amplitudes(s, M, 1.2) for s in (71, 72)])
    z = W.phase_draws([1, 0, 2, 0, 0, 1, 0, 1, 0, 0], range(5, 21))
    psi = fh.init_fieldnumber(b, z[0])
    res = fh.evolve_rk4(model, b, psi, dt, 60, every=30)
    ref, recs = _oracle_run(orc, states.fieldnumber_state(orc, z[0]), dt, 60, 30)
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(M, res, recs)
    psi = fh.init_fieldnumber(b, z[0])
    fh.evolve_taylor2(model, b, psi, dt, 40, c2=0.5)
    ref2, _ = evolve.taylor2(orc, states.fieldnumber_state(orc, z[0]), dt, 40, c2=0.5)
    assert np.linalg.norm(psi.cpu().numpy() - ref2) <= 1e-10
    both = fh.init_fieldnumber(b, z)
    fh.evolve_rk4(model, b, both, dt, 25)
    for q in (0, 7, 15):
        one = fh.init_fieldnumber(b, z[q])
        fh.evolve_rk4(model, b, one, dt, 25)
        assert torch.equal(both[:, q].contiguous(), one)
    ref3 = evolve.adjoint(orc, states.fieldnumber_state(orc, z[1]), dt, 20, evolve.objective_PO(orc))
    adj = fh.adjoint_rk4(model, b, fh.init_fieldnumber(b, z[1]), dt, 20, 6, fh.FH_J_PO)
    assert abs(adj["J"][0] - ref3["J"]) <= 1e-10
    assert abs(adj["dLambda"][0] - ref3["dLambda"]) <= 1e-9 * max(1, abs(ref3["dLambda"]))
    del al


def test_tangent_at_zero_interaction():
    """Lambda = 0 takes the tangent's other branch (G y as its own application):
    dJ/dLambda at Lambda = 0 against the oracle's adjoint and the GPU adjoint."""
    M, dt, nsteps = 4, 5e-3, 20
    sectors = W.all_sectors(M, 8)
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    orc, model, b = _pair(M, sectors, omega, 0.0, V)
    alpha = W.coherent_amplitudes(33, M, 1.4)
    ref = evolve.adjoint(orc, states.coherent_state(orc, alpha), dt, nsteps, evolve.objective_Q(orc))
    tan = fh.tangent_rk4(model, b, fh.init_coherent(b, alpha), dt, nsteps, fh.FH_J_Q)
    adj = fh.adjoint_rk4(model, b, fh.init_coherent(b, alpha), dt, nsteps, 5, fh.FH_J_Q)
    assert abs(tan["dLambda"][0] - ref["dLambda"]) <= 1e-9 * max(1, abs(ref["dLambda"]))
    assert abs(tan["dLambda"][0] - adj["dLambda"][0]) <= 1e-10 * max(1, abs(adj["dLambda"][0]))


# ------------------------------------------------ the benchmark's instantiation --
@pytest.mark.timeout(600)
def test_rk4_benchmark_instantiation_m8():
    """The fused RK4 stages at M = 8 (the kernels the benchmark times) against
    the oracle: the benchmark's frequencies, long-range V, Lambda, dt and
    launch walk (one contiguous eighth of the tiles per XCD) on the M = 8,
    N = 18, P = 0 sector (60,115 states), 40 steps, records every 20.  One
    column: the number state of the benchmark's draw rule and a random vector,
    each against the oracle; 2, 4 and 8 columns (eight distinct vectors) bitwise
    equal to one-column runs of the same vectors."""
    import os

    wl = W.large_sector()
    M, N, dt, nsteps, every = wl.M, 18, wl.dt, 40, 20
    sectors = [(N, 0)]
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    orc = Oracle(M, M, wl.omega, wl.Lambda, wl.V, sectors, threads=threads)
    model, b = fh.Model(M, wl.omega, wl.Lambda, wl.V), fh.Basis(M, sectors)
    assert b.total == orc.total == 60_115
    b.set_launch(0, 2)
    occ = W.random_occupations_in_sector(2, N, M, 0)
    cols = [states.number_state(orc, occ)]
    for q in range(1, 8):
        x = W.random_psi(b.total, 500 + q)
        cols.append(x / np.linalg.norm(x))
    singles = []
    for q, x in enumerate(cols):
        psi = torch.from_numpy(x).cuda()
        res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=every)
        singles.append(psi)
        if q < 2:
            ref, recs = _oracle_run(orc, x, dt, nsteps, every)
            assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10, q
            _check_records(M, res, recs)
    for nrhs in (2, 4, 8):
        psi = torch.from_numpy(np.ascontiguousarray(np.stack(cols[:nrhs], axis=1))).cuda()
        fh.evolve_rk4(model, b, psi, dt, nsteps)
        for q in range(nrhs):
            assert torch.equal(psi[:, q].contiguous(), singles[q]), (nrhs, q)


def test_squeezing_of_a_site_kerr_state_on_gpu():
    """fh_derive on GPU moments of an evolved multi-mode state (the pinned state
    of S3: contact V, w = 0, one occupied site mode b_1 of M = 4): V_- of the
    principal mode and per mode against the oracle run, and V_- against the
    single-mode Kerr closed form within RK4's truncation error."""
    import math

    import os

    M, Lam, x, Nmax, dt, nsteps, every = 4, 0.3, 1, 14, 1e-3, 600, 200
    F = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M) / math.sqrt(M)
    beta = np.zeros(M, np.complex128)
    beta[x] = 0.8 * np.exp(0.7j)
    alpha = F.conj().T @ beta
    sectors = W.all_sectors(M, Nmax)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    orc = Oracle(M, M, np.zeros(M), Lam, W.V_contact(M), sectors, threads=threads)
    model, b = fh.Model(M, np.zeros(M), Lam, W.V_contact(M)), fh.Basis(M, sectors)
    psi = fh.init_coherent(b, alpha)
    res = fh.evolve_rk4(model, b, psi, dt, nsteps, every=every)
    ref, recs = _oracle_run(orc, states.coherent_state(orc, alpha), dt, nsteps, every)
    assert np.linalg.norm(psi.cpu().numpy() - ref) <= 1e-10
    _check_records(M, res, recs)
    for r, rec in enumerate(res.records[:, 0]):
        t = r * every * dt
        g = fh.derive(M, *fh.unpack_moments(M, rec))
        n = abs(beta[x]) ** 2
        m1 = beta[x] * np.exp(n * (np.exp(-1j * Lam * M * t) - 1))
        m2 = beta[x] ** 2 * np.exp(-1j * Lam * M * t) * np.exp(n * (np.exp(-2j * Lam * M * t) - 1))
        want = 1.0 + 2.0 * (n - abs(m1) ** 2) - 2.0 * abs(m2 - m1 * m1)
        assert abs(g["vminus"] - want) <= 1e-8, (t, g["vminus"], want)


def test_tangent_at_tiny_interaction():
    """At a tiny nonzero Lambda the tangent takes G y by its own application
    (deriving it from H y would cost eps |omega.n| / |Lambda G| of accuracy):
    dJ/dLambda at Lambda = 1e-8 against the oracle's adjoint and the GPU
    adjoint."""
    M, dt, nsteps, Lam = 4, 5e-3, 20, 1e-8
    sectors = W.all_sectors(M, 8)
    omega, V = W.omega_quadratic(M), W.V_longrange(M)
    orc, model, b = _pair(M, sectors, omega, Lam, V)
    alpha = W.coherent_amplitudes(33, M, 1.4)
    ref = evolve.adjoint(orc, states.coherent_state(orc, alpha), dt, nsteps, evolve.objective_Q(orc))
    tan = fh.tangent_rk4(model, b, fh.init_coherent(b, alpha), dt, nsteps, fh.FH_J_Q)
    adj = fh.adjoint_rk4(model, b, fh.init_coherent(b, alpha), dt, nsteps, 5, fh.FH_J_Q)
    assert abs(tan["dLambda"][0] - ref["dLambda"]) <= 1e-9 * max(1, abs(ref["dLambda"]))
    assert abs(tan["dLambda"][0] - adj["dLambda"][0]) <= 1e-10 * max(1, abs(adj["dLambda"][0]))


@pytest.mark.parametrize("which", ["large_sector", "fieldnumber_draw"])
def test_rk4_steps_full_size(which):
    """Full size, in the benchmark's launch configuration (basis default:
    counter walk, every workgroup the CU holds; FH_TIMING): the one large
    sector (M=8, N=48, P=0, 25.4M states) and one field-number draw (M=10,
    N=30, all P, 212M states), one column.  Sampled rows of a plain H psi
    launch (APPLY) against the oracle; then two fused RK4 steps (FIRST, MID,
    MID, LAST epilogues) against the classical RK4 combination of APPLY
    launches, to rounding; the moments recorded after the last step equal
    those of the composed state."""
    w = W.large_sector() if which == "large_sector" else W.fieldnumber_draws(16, 30)
    orc = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    b = fh.Basis(w.M, w.sectors)
    assert b.total == orc.total
    x0 = W.periodic_psi(b.total, 23)
    x0 /= np.linalg.norm(x0)
    rows = _sample_rows(orc, np.random.default_rng(17), 2000)
    x = torch.from_numpy(x0).cuda()
    hx = fh.apply_h(model, b, x)
    want = orc.apply_h_rows(x0, rows)
    assert np.abs(hx[torch.from_numpy(rows).cuda()].cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()
    del hx, x0, orc
    psi = x.clone()
    res = fh.evolve_rk4(model, b, psi, w.dt, 2, every=1, flags=fh.FH_TIMING)
    y = x
    for _ in range(2):
        k1 = -1j * fh.apply_h(model, b, y)
        k2 = -1j * fh.apply_h(model, b, y + (w.dt / 2) * k1)
        k3 = -1j * fh.apply_h(model, b, y + (w.dt / 2) * k2)
        k4 = -1j * fh.apply_h(model, b, y + w.dt * k3)
        y = y + (w.dt / 6) * (k1 + 2 * k2 + 2 * k3 + k4)
        del k1, k2, k3, k4
    assert float(torch.linalg.vector_norm(psi - y)) <= 1e-13
    # the moments recorded after the last step equal those of the composed state
    assert len(res.records) == 3
    n2, a, Mm, A = fh.unpack_moments(w.M, res.records[-1, 0])
    wn2, wa, wM, wA = fh.moments(b, y)
    assert abs(n2 - wn2) <= 1e-13
    for g_, w_ in ((a, wa), (Mm, wM), (A, wA)):
        assert np.abs(np.asarray(g_) - np.asarray(w_)).max() <= 1e-10 * max(1.0, np.abs(np.asarray(w_)).max())


def test_adjoint_chunked_correlators_on_the_benchmark_sector():
    """The correlators of the adjoint at M >= 8 run over chunks of 2^24 rows;
    the benchmark's sector (25.4M states) spans two.  dJ/dLambda of the
    adjoint (which sums the correlators) against the forward-mode tangent
    (which does not use them) and against a central difference of GPU forward
    runs, for J = <n_0>(T) after 3 steps from a seeded vector."""
    w = W.large_sector()
    model = fh.Model(w.M, w.omega, w.Lambda, w.V)
    b = fh.Basis(w.M, w.sectors)
    assert b.total > (1 << 24)
    x = torch.from_numpy(W.periodic_psi(b.total, 29)).cuda()
    x /= torch.linalg.vector_norm(x)
    dt, nsteps = w.dt, 3
    adj = fh.adjoint_rk4(model, b, x, dt, nsteps, nsteps, fh.FH_J_NMODE, 0)
    tan = fh.tangent_rk4(model, b, x, dt, nsteps, fh.FH_J_NMODE, 0)
    assert abs(adj["J"][0] - tan["J"][0]) <= 1e-12 * abs(tan["J"][0])
    assert abs(adj["dLambda"][0] - tan["dLambda"][0]) <= 1e-10 * abs(tan["dLambda"][0])
    # J ~ 6 is summed to ~1e-15 relative, so the step must keep that rounding
    # (6e-15 / 2h) well under the tolerance
    h = 1e-2 * abs(w.Lambda)
    Jpm = []
    for sgn in (1, -1):
        m2 = fh.Model(w.M, w.omega, w.Lambda + sgn * h, w.V)
        Jpm.append(float(fh.adjoint_rk4(m2, b, x, dt, nsteps, nsteps, fh.FH_J_NMODE, 0)["J"][0]))
    cd = (Jpm[0] - Jpm[1]) / (2 * h)
    assert abs(adj["dLambda"][0] - cd) <= 1e-5 * abs(cd)


@pytest.mark.parametrize("M,N", [(7, 48), (9, 28)])
def test_counter_walk_kernels_m7_m9(M, N):
    """The counter-walk stage kernels of M = 7 and 9, which no benchmark
    workload runs: one sector (N, P = 0) of 3.7M / 3.4M states, enough that
    every workgroup takes at least 16 tiles.  Sampled rows of H psi against
    the oracle; two fused RK4 steps against the RK4 combination of plain H psi
    launches."""
    omega, V, Lam, dt = W.omega_quadratic(M), W.V_longrange(M), 0.02, 5e-4
    orc = Oracle(M, M, omega, Lam, V, [(N, 0)])
    model, b = fh.Model(M, omega, Lam, V), fh.Basis(M, [(N, 0)])
    assert b.total == orc.total and b.total // 256 >= 16 * 768
    x0 = W.periodic_psi(b.total, 31 + M)
    x0 /= np.linalg.norm(x0)
    rows = _sample_rows(orc, np.random.default_rng(M), 1500)
    x = torch.from_numpy(x0).cuda()
    hx = fh.apply_h(model, b, x)
    want = orc.apply_h_rows(x0, rows)
    assert np.abs(hx[torch.from_numpy(rows).cuda()].cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()
    del hx, x0, orc
    psi = x.clone()
    fh.evolve_rk4(model, b, psi, dt, 2)
    y = x
    for _ in range(2):
        k1 = -1j * fh.apply_h(model, b, y)
        k2 = -1j * fh.apply_h(model, b, y + (dt / 2) * k1)
        k3 = -1j * fh.apply_h(model, b, y + (dt / 2) * k2)
        k4 = -1j * fh.apply_h(model, b, y + dt * k3)
        y = y + (dt / 6) * (k1 + 2 * k2 + 2 * k3 + k4)
    assert float(torch.linalg.vector_norm(psi - y)) <= 1e-13


@pytest.mark.parametrize("nrhs", [2, 4])
def test_counter_walk_multi_column_bitwise(nrhs):
    """Several columns under the counter walk (M = 8, N = 40, P = 0: 7.9M
    states, every workgroup taking many tile passes): two fused RK4 steps of
    an nrhs-column vector equal, column by column and bit for bit, the same
    steps of each column alone."""
    M = 8
    w = W.large_sector()
    model, b = fh.Model(M, w.omega, w.Lambda, w.V), fh.Basis(M, [(40, 0)])
    assert b.total > 7_000_000
    cols = [W.periodic_psi(b.total, 40 + q) for q in range(nrhs)]
    X = torch.from_numpy(np.stack(cols, axis=1)).cuda().contiguous()
    fh.evolve_rk4(model, b, X, w.dt, 2)
    for q in range(nrhs):
        one = torch.from_numpy(cols[q]).cuda()
        fh.evolve_rk4(model, b, one, w.dt, 2)
        assert torch.equal(X[:, q].contiguous(), one), q
