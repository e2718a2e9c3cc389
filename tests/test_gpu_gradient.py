"""Adjoint (gradient) kernel on the GPU against the oracle's dual-number gradient, against central
differences of the GPU's own forward energies, the translation sum rule, and through the
torch.autograd.Function."""
import numpy as np
import pytest

import helpers
import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as m
    m.load_library()
    return m


def gpu_grad(shgo, b, n, D, screen=0.0):
    dn, dc, e = shgo.nuclear_attraction_grad(b, n, D, screen)
    return dn.cpu().numpy(), dc.cpu().numpy(), float(e.cpu().numpy()[0])


def assert_grad(got, ref, what):
    dn, dc, E = got
    rn, rc, rE = ref
    scale = max(np.abs(rn).max(initial=0.0), np.abs(rc).max(initial=0.0), 1e-300)
    for name, x, y in (("nuclei", dn, rn), ("centers", dc, rc)):
        err = np.abs(x - y)
        bad = err > RTOL * np.abs(y) + 1e-12 * scale
        assert not bad.any(), f"{what} {name}: {int(bad.sum())} off, max err {err.max():.3e} (scale {scale:.3e})"
    assert E == pytest.approx(rE, rel=1e-11, abs=1e-12)


def test_small_molecule_against_oracle(shgo):
    b, n = synth.small_molecule(seed=1)
    D = synth.density(b.nbf(), seed=5)
    assert_grad(gpu_grad(shgo, b, n, D), oracle.grad(b, n, D), "small molecule")


def test_every_class_against_oracle(shgo):
    b, n = synth.molecule(seed=51, n_atoms=3, box=4.0, ls=(0, 1, 2, 3, 4, 5, 6), kmax=2)
    D = synth.density(b.nbf(), seed=6)
    assert_grad(gpu_grad(shgo, b, n, D), oracle.grad(b, n, D), "l <= 6")


def test_nonsymmetric_density_and_shared_centers(shgo):
    # D need not be symmetric; shells of one atom share a center (R = 0 pairs)
    b, n = synth.molecule(seed=52, n_atoms=2, box=3.0, ls=(0, 1, 2, 3), kmax=3)
    D = np.random.default_rng(3).normal(0, 0.2, (b.nbf(), b.nbf()))
    assert_grad(gpu_grad(shgo, b, n, D), oracle.grad(b, n, D), "nonsymmetric D")


def test_screened_contracted_molecule(shgo):
    b, n = synth.molecule(seed=53, n_atoms=8, box=8.0, ls=(0, 1, 2, 3), kmax=6)
    D = synth.density(b.nbf(), seed=7)
    screen = 1e-12
    assert_grad(gpu_grad(shgo, b, n, D, screen), oracle.grad(b, n, D, screen), "screened")


def test_sparse_molecule_with_fully_screened_pairs(shgo):
    # a sparse molecule where many shell pairs keep no primitive pair: those pairs add nothing
    b, n = synth.molecule(seed=54, n_atoms=10, box=14.0, ls=(0, 1, 2, 3), kmax=5)
    D = synth.density(b.nbf(), seed=11)
    pa, pb = synth.all_pairs(b.n_shells)
    R2 = np.sum((b.center[pa] - b.center[pb]) ** 2, axis=1)
    for screen in (1e-12, 1e-8):
        empty = 0
        for i in range(len(pa)):
            ea = b.expo[b.prim_off[pa[i]]:b.prim_off[pa[i]] + b.nprim[pa[i]]]
            eb = b.expo[b.prim_off[pb[i]]:b.prim_off[pb[i]] + b.nprim[pb[i]]]
            mu = ea[:, None] * eb[None, :] / (ea[:, None] + eb[None, :])
            empty += not np.any(np.exp(-mu * R2[i]) > screen)
        assert empty > len(pa) // 5
        assert_grad(gpu_grad(shgo, b, n, D, screen), oracle.grad(b, n, D, screen), f"sparse, screen {screen}")


def test_many_nuclei_span_several_lane_rounds(shgo):
    # 150 nuclei: three rounds of the 64-lane nucleus loop, the last one ragged
    b, _ = synth.molecule(seed=54, n_atoms=2, box=3.0, ls=(1, 2), kmax=2)
    rng = np.random.default_rng(54)
    n = synth.Nuclei(rng.uniform(-3, 6, (150, 3)), rng.integers(1, 9, 150).astype(np.float64))
    D = synth.density(b.nbf(), seed=8)
    assert_grad(gpu_grad(shgo, b, n, D), oracle.grad(b, n, D), "150 nuclei")


def test_long_contractions(shgo):
    # shell pairs of 256 to 400 primitive pairs (the pair key saturates), screened and not
    b, n = synth.long_contractions(seed=71)
    D = synth.density(b.nbf(), seed=8)
    for screen in (0.0, 1e-6):
        assert_grad(gpu_grad(shgo, b, n, D, screen), oracle.grad(b, n, D, screen=screen), f"K up to 20, screen {screen}")


def test_central_differences_of_gpu_energies(shgo):
    import torch
    b, n = synth.molecule(seed=55, n_atoms=6, box=6.0, ls=(0, 1, 2, 3), kmax=4)
    D = synth.density(b.nbf(), seed=9)
    Dt = torch.as_tensor(D, device="cuda")
    dn, dc, _ = gpu_grad(shgo, b, n, D)

    def energy(bb, nn):
        V = shgo.nuclear_attraction(bb, nn)
        return float((V * Dt).sum().item())

    h = 1e-4
    rng = np.random.default_rng(10)
    for _ in range(6):
        c, x = int(rng.integers(n.n)), int(rng.integers(3))
        pp, pm = n.pos.copy(), n.pos.copy()
        pp[c, x] += h
        pm[c, x] -= h
        fd = (energy(b, synth.Nuclei(pp, n.Z)) - energy(b, synth.Nuclei(pm, n.Z))) / (2 * h)
        assert fd == pytest.approx(dn[c, x], rel=1e-6, abs=1e-8)
        s = int(rng.integers(b.n_shells))
        cp, cm = b.center.copy(), b.center.copy()
        cp[s, x] += h
        cm[s, x] -= h
        bp = synth.Basis(cp, b.l, b.nprim, b.prim_off, b.expo, b.coef)
        bm = synth.Basis(cm, b.l, b.nprim, b.prim_off, b.expo, b.coef)
        fd = (energy(bp, n) - energy(bm, n)) / (2 * h)
        assert fd == pytest.approx(dc[s, x], rel=1e-6, abs=1e-8)


def test_translation_sum_rule(shgo):
    b, n = synth.molecule(seed=56, n_atoms=20, box=10.0, ls=(0, 1, 2, 3), kmax=6)
    D = synth.density(b.nbf(), seed=11)
    dn, dc, _ = gpu_grad(shgo, b, n, D, 1e-12)
    total = dn.sum(axis=0) + dc.sum(axis=0)
    assert np.abs(total).max() <= 1e-10 * np.abs(np.concatenate([dn, dc])).max()


def test_full_size_gradient_properties(shgo):
    """The 500-atom gradient workload at full size (nbf 8000, screened 1e-12), where the oracle is
    too slow: E against sum D V of the GPU forward, the translation sum rule, and central
    differences (h = 1e-4) of the GPU's own energies for 12 nuclear and 12 shell-center coordinates,
    within 1e-6 of the gradient vector's norm.
    Each difference takes only the partial sum a displacement changes: for a nucleus, E of that
    nucleus alone over the shell pairs that keep a primitive pair; for a shell center, the blocks of
    that shell's pairs (pair list frozen at the reference geometry)."""
    import torch
    b, n = synth.gradient_molecule(seed=5)
    D = synth.density(b.nbf(), seed=5)
    screen = 1e-12
    dn, dc, E = gpu_grad(shgo, b, n, D, screen)
    total = dn.sum(axis=0) + dc.sum(axis=0)
    assert np.abs(total).max() <= 1e-10 * np.abs(np.concatenate([dn, dc])).max()
    Dt = torch.as_tensor(D, device="cuda")
    V = shgo.nuclear_attraction(b, n, screen=screen)
    assert float((V.view(-1) * Dt.view(-1)).sum().item()) == pytest.approx(E, rel=1e-12)
    del V
    off = b.shell_offsets()
    pa, pb = synth.all_pairs(b.n_shells)
    kept = helpers.surviving_prim_pairs(b, pa, pb, screen) > 0

    def dweights(qa, qb):
        # E's weight of each block entry V[a, b]: D[a, b] + D[b, a]^T off the diagonal, D[a, a] on it
        out = []
        for a, c in zip(qa, qb):
            ra, rc = slice(off[a], off[a] + 2 * b.l[a] + 1), slice(off[c], off[c] + 2 * b.l[c] + 1)
            w = D[ra, rc] + (D[rc, ra].T if a != c else 0.0)
            out.append(w.ravel())
        return torch.as_tensor(np.concatenate(out), device="cuda")

    def partial(bb, nn, qa, qb, w):
        blocks = shgo.nuclear_attraction_pairs(bb, nn, qa, qb, screen=screen)
        return float((blocks * w).sum().item())

    def fd_ok(fd, g, x, what):
        # the central difference's truncation error, h^2/6 times a third derivative, scales with
        # the size of the whole gradient vector of that nucleus or shell, not with one component
        assert abs(fd - g[x]) <= 1e-6 * np.linalg.norm(g) + 1e-8, (what, fd, g)

    h = 1e-4
    rng = np.random.default_rng(12)
    qa, qb = pa[kept], pb[kept]
    w_all = dweights(qa, qb)
    for c in rng.choice(n.n, 12, replace=False):
        x = int(rng.integers(3))
        pp, pm = n.pos[c:c + 1].copy(), n.pos[c:c + 1].copy()
        pp[0, x] += h
        pm[0, x] -= h
        ep = partial(b, synth.Nuclei(pp, n.Z[c:c + 1]), qa, qb, w_all)
        em = partial(b, synth.Nuclei(pm, n.Z[c:c + 1]), qa, qb, w_all)
        fd_ok((ep - em) / (2 * h), dn[c], x, ("nucleus", c, x))
    for s_ in rng.choice(b.n_shells, 12, replace=False):
        x = int(rng.integers(3))
        mine = (qa == s_) | (qb == s_)
        sa, sb = qa[mine], qb[mine]
        w = dweights(sa, sb)
        es = []
        for sign in (1.0, -1.0):
            cen = b.center.copy()
            cen[s_, x] += sign * h
            es.append(partial(synth.Basis(cen, b.l, b.nprim, b.prim_off, b.expo, b.coef), n, sa, sb, w))
        fd_ok((es[0] - es[1]) / (2 * h), dc[s_], x, ("center", s_, x))


def test_autograd_function(shgo):
    import torch
    b, n = synth.small_molecule(seed=2)
    D = torch.as_tensor(synth.density(b.nbf(), seed=12), device="cuda")
    centers = torch.tensor(b.center, device="cuda", requires_grad=True)
    pos = torch.tensor(n.pos, device="cuda", requires_grad=True)
    V = shgo.NuclearAttractionFn.apply(centers, pos, b, n.Z, 0.0)
    ref = oracle.nuc_matrix(b, n)
    assert np.allclose(V.detach().cpu().numpy(), ref, rtol=1e-11, atol=1e-13)
    (V * D).sum().backward()
    rn, rc, _ = oracle.grad(b, n, D.cpu().numpy())
    assert np.allclose(pos.grad.cpu().numpy(), rn, rtol=RTOL, atol=1e-12 * np.abs(rn).max())
    assert np.allclose(centers.grad.cpu().numpy(), rc, rtol=RTOL, atol=1e-12 * np.abs(rc).max())


def test_gradient_edge_cases(shgo):
    import torch
    b, n = synth.small_molecule(seed=1)
    D = synth.density(b.nbf(), seed=5)
    # no nuclei: E = 0 and every gradient vanishes
    empty = synth.Nuclei(np.zeros((0, 3)), np.zeros(0))
    dn, dc, E = gpu_grad(shgo, b, empty, D)
    assert dn.shape == (0, 3) and not dc.any() and E == 0.0
    # a pair plan is refused
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_pairs(ctx, b, n, [0], [1])
    with pytest.raises(shgo.ShgoError) as e:
        z = torch.zeros(1, dtype=torch.float64, device="cuda")
        shgo.shgo_execute_grad(plan, torch.zeros((b.nbf(), b.nbf()), dtype=torch.float64, device="cuda"),
                               torch.zeros((n.n, 3), dtype=torch.float64, device="cuda"),
                               torch.zeros((b.n_shells, 3), dtype=torch.float64, device="cuda"), z)
    assert e.value.status == shgo.SHGO_ERR_INVALID_ARG
