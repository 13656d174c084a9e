"""Parity at the benchmark's full sizes, in its launch configuration (filter
blocks of 128 vectors), on outputs the oracle can afford: sampled columns of
Htilde X, and residuals of sampled Ritz pairs recomputed on the CPU."""
import numpy as np
import pytest

from oracle import fem
import workload
from gpu_util import make_ctx, oracle_apply

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["large_p6", "large_p5"])
def test_apply_full_size_sampled_columns(name):
    import torch
    prob = workload.PROBLEMS[name]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block_device(prob.n_dof, prob.block_width, prob.x0_seed, device="cuda:0")
    Y = c.apply(X)
    cols = [0, 37, 64, prob.block_width - 1]          # both 64-column tiles, first and last column
    Xs = X[:, cols].cpu().numpy()
    Ys = Y[:, cols].cpu().numpy()
    Yo = oracle_apply(prob.L, prob.n_el, prob.p, V)(Xs)
    rel = np.max(np.abs(Ys - Yo)) / np.max(np.abs(Yo))
    assert rel < 1e-13, rel
    # reduced-precision paths on the same block, per output against a bound
    # from the format's unit roundoff: |dY_i| <= (k u + n_loc u32) (|H||x|)_i
    # (k = 3 covers the rounding of both BF16 operands, or the dropped lo*lo
    # term of the split; n_loc u32 the FP32 accumulation)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    HabsX = fem.apply_kron(np.abs(A), np.abs(V), np.abs(Xs))
    n_loc = (prob.p + 1) ** 3
    u32 = 2.0 ** -24
    for prec, u, floor in (("fp32", u32, 0.0), ("bf16", 2.0 ** -8, 1e-4), ("bf16x3", 2.0 ** -16, 1e-8)):
        Yp = c.apply(X, prec=prec)[:, cols].cpu().numpy()
        err = np.abs(Yp - Yo)
        bound = (3.0 * u + n_loc * u32) * HabsX
        assert np.all(err <= bound), (prec, np.max(err / bound))
        # and the reduced format really ran (its error is above FP64 level)
        assert np.max(err / HabsX) > floor, (prec, np.max(err / HabsX))
    del X, Y
    torch.cuda.empty_cache()
    c.close()


def _ho_levels(L, n_el, p, om, count):
    """Exact discrete eigenvalues of the separable harmonic-oscillator operator:
    sums of three eigenvalues of the 1D operator with the 1D potential."""
    A = fem.operator_1d(L, n_el, p)
    x = fem.node_coords_1d(L, n_el, p)[1:-1]
    a = np.linalg.eigvalsh(A + np.diag(0.5 * om * om * (x - L / 2) ** 2))[:12]
    return np.sort((a[:, None, None] + a[None, :, None] + a[None, None, :]).reshape(-1))[:count]


@pytest.mark.parametrize("name,ladder,mixed", [("large_p6", ("fp64",), False),
                                               ("large_p6", ("bf16", "fp32", "fp64"), True),
                                               ("large_p5", ("fp64",), False)])
def test_solve_harmonic_oscillator_at_full_mesh_shape(name, ladder, mixed):
    """The full solve on the workload's mesh (24^3 cells p = 6, or 32^3 cells
    p = 5) with V = 1/2 |x - L/2|^2 (separable, so the exact discrete
    eigenvalues are sums of 1D ones): the lowest 56 states (the shells
    n = 0..5 of omega (n + 3/2), a cluster boundary) to 1e-10 relative on the
    FP64 path; on the BF16 -> FP32 -> FP64 ladder with the mixed CholGS to the
    1e-6 Ha residual target (a residual bounds the eigenvalue error)."""
    import torch
    prob = workload.PROBLEMS[name]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, V=None)
    V = workload.harmonic(c.dof_coords(), 1.0, [prob.L / 2] * 3)
    c.set_potential(V)
    N = 56
    ref = _ho_levels(prob.L, prob.n_el, prob.p, 1.0, N + 1)
    assert ref[N] - ref[N - 1] > 0.5                   # the shell boundary
    nb = workload.block_size(N)
    X = workload.start_block_device(prob.n_dof, nb, 91, device="cuda:0")
    fp64 = ladder == ("fp64",)
    tol = 1e-9 * max(1.0, abs(ref[0])) if fp64 else 1e-6
    out = c.solve(X, N, prob.degree, tol, max_iter=200, ladder=ladder, mixed_cholgs=mixed)
    assert out["converged"], out
    err = np.abs(out["evals"][:N] - ref[:N])
    if fp64:
        assert np.max(err / np.maximum(np.abs(ref[:N]), 1.0)) < 1e-10, err
    else:
        assert np.max(err) < 1e-6, err
    cols = [0, 9, 20, 55]
    Xs = X[:, cols].cpu().numpy()
    r_cpu = np.linalg.norm(oracle_apply(prob.L, prob.n_el, prob.p, V)(Xs) - Xs * out["evals"][cols][None, :], axis=0)
    np.testing.assert_allclose(out["resid"][cols], r_cpu, rtol=1e-6, atol=1e-12)
    del X
    torch.cuda.empty_cache()
    c.close()


def test_residual_certificate_full_size_large_p6():
    """Two passes of the solve on the full 568-vector block; for sampled Ritz
    pairs the residual ||Htilde x - lambda x|| recomputed on the CPU from the
    GPU's vectors equals the reported one, and the vectors are orthonormal."""
    import torch
    prob = workload.PROBLEMS["large_p6"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device="cuda:0")
    out = c.solve(X, prob.nstates, prob.degree, 1e-30, max_iter=2, block_width=prob.block_width)
    assert out["iters"] == 2
    cols = [0, 1, 100, 511, 567]
    Xs = X[:, cols].cpu().numpy()
    G = Xs.T @ Xs
    assert np.max(np.abs(G - np.eye(len(cols)))) < 1e-12
    lam = out["evals"][cols]
    r_cpu = np.linalg.norm(oracle_apply(prob.L, prob.n_el, prob.p, V)(Xs) - Xs * lam[None, :], axis=0)
    np.testing.assert_allclose(out["resid"][cols], r_cpu, rtol=1e-8, atol=1e-11)
    # Rayleigh quotients of the CPU operator reproduce the Ritz values
    rq = np.einsum("ij,ij->j", Xs, oracle_apply(prob.L, prob.n_el, prob.p, V)(Xs))
    np.testing.assert_allclose(rq, lam, rtol=0, atol=1e-10 * max(1.0, np.max(np.abs(lam))))
    del X
    torch.cuda.empty_cache()
    c.close()


def test_density_full_size_large_p5():
    """Spectrum-splitting RR (out of place, N_fr = 15 % of N) and the density
    on the full large_p5 block: the particle count over all 4.0M nodes, and
    sampled nodes recomputed on the CPU from the GPU's own rows."""
    import torch
    import paper_1903_10959_amd as P
    from oracle import density as ode
    prob = workload.PROBLEMS["large_p5"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device="cuda:0")
    c.orthonormalize(X)
    n_fr = int(round(0.15 * prob.nstates))
    n_oc = prob.nblock - n_fr
    Xfr = torch.empty((prob.n_dof, n_fr), dtype=torch.float64, device="cuda:0")
    ev, _ = c.rayleigh_ritz_split(X, n_fr, mixed=True, Xfr=Xfr)
    ne = 2 * (n_oc + 0.5 * n_fr)
    sigma = 1.58e-3                                  # k_B T at 500 K, in Ha
    mu = P.fermi_level(ev, n_oc, ne, sigma)
    rho = c.density(X, Xfr, ev, mu, sigma)
    M = torch.from_numpy(fem.mass_diag_kron(prob.L, prob.n_el, prob.p)).to("cuda:0")
    count = float(torch.sum(M * rho))
    assert abs(count - ne) < 1e-9 * ne, (count, ne)
    rows = np.array([0, 1, 12345, prob.n_dof // 2, prob.n_dof - 1])
    idx = torch.from_numpy(rows).to("cuda:0")
    minv = 1.0 / np.sqrt(M[idx].cpu().numpy())
    r_cpu = ode.density_split(X[idx].cpu().numpy(), Xfr[idx].cpu().numpy(), ev, mu, sigma, minv)
    np.testing.assert_allclose(rho[idx].cpu().numpy(), r_cpu, rtol=1e-13, atol=0)
    del X, Xfr, rho, M
    torch.cuda.empty_cache()
    c.close()


def test_apply_complex_full_size_sampled_columns():
    """The complex Bloch operator on a periodic cell with the large_p6 element
    size (24^3 cells, p = 6: 144^3 = 2,985,984 DoFs), 64 complex columns (two
    column tiles of the kernel); sampled columns against the oracle's
    Kronecker-sum apply."""
    import torch
    import paper_1903_10959_amd as P
    from oracle import kpoint
    L, n_el, p = 40.0, 24, 6
    k = np.array([0.05, 0.11, -0.08])
    c = P.Context(0).set_mesh(L, n_el, p, periodic=True)
    V = workload.eval_wells(workload.draw_wells(64, L, 2, (1.0, 3.0), (0.5, 1.5)), c.dof_coords())
    c.set_potential(V)
    c.set_kpoint(k)
    g = torch.Generator(device="cuda:0").manual_seed(77)
    X = torch.randn((c.n_dof, 64), dtype=torch.complex128, device="cuda:0", generator=g)
    Y = c.apply_complex(X)
    cols = [0, 31, 32, 63]
    Xs = X[:, cols].cpu().numpy()
    A = [kpoint.operator_1d_periodic(L, n_el, p, kd) for kd in k]
    Yo = kpoint.apply_kron_k(*A, V, Xs)
    rel = np.max(np.abs(Y[:, cols].cpu().numpy() - Yo)) / np.max(np.abs(Yo))
    assert rel < 1e-13, rel
    del X, Y
    torch.cuda.empty_cache()
    c.close()


def test_poisson_full_size_large_p6_mesh():
    """Jacobi-PCG on the large_p6 mesh (2,924,207 DoFs): the relative residual
    of the returned potential, recomputed on the CPU through the oracle's
    Kronecker form of the operator, meets the tolerance."""
    import torch
    import paper_1903_10959_amd as P
    from oracle import poisson
    prob = workload.PROBLEMS["large_p6"]
    c = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    xyz = c.dof_coords()
    rho = -workload.eval_wells(workload.problem_wells(prob), xyz)
    out = c.poisson_solve(torch.from_numpy(rho).to("cuda:0"), charges=[(123456, -4.0)], tol=1e-10)
    assert out["converged"]
    phi = out["phi"].cpu().numpy()
    M = fem.mass_diag_kron(prob.L, prob.n_el, prob.p)
    A1 = fem.operator_1d(prob.L, prob.n_el, prob.p)
    sq = np.sqrt(M)
    Aphi = sq * fem.apply_kron(A1, np.zeros_like(phi), sq * phi) / (2 * np.pi)   # K_half / (2 pi)
    f = poisson.load_vector(M, rho, [123456], [-4.0])
    rel = np.linalg.norm(f - Aphi) / np.linalg.norm(f)
    assert rel < 2e-10, rel
    c.close()
