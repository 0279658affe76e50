"""GPU: the discontinuous P1 space (dof 3 t + a) and the hypersingular
operator assembled through the single layer on it (Eq. hyp_via_slp).

  * DP1 entries of the Laplace and Helmholtz single, double and adjoint
    double layer against the oracle, FP64 (1e-11) and FP32 (Laplace single
    layer 1e-5 entrywise, others 1e-5 / 1e-4 normwise), ragged shapes;
  * DP1 singular pairs: each entry is one pair's local matrix element, against
    the oracle's P1 local matrices;
  * the hypersingular H-matrix through the DP1 single layer, FP32 and FP64,
    regular part (dense_mode 1): matvec against the oracle's direct P1
    hypersingular matrix on the same pairs within the ACA tolerance's reach
    (the same relative bar as the single layer: 1e-5 at ACA tol 1e-6);
  * complete (dense_mode 2): the unit sphere's degree-1 eigenvalue 2/3;
  * on the level-6 icosphere, FP32 ACA ranks of the DP1 single layer within
    1.2x of FP64 (direct FP32 hypersingular entries lose (r/h)^2 in relative
    accuracy and ACA on them does not converge at tol 1e-5).
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ico3():
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    yield xyz, tri, mesh, O.OracleMesh(xyz, tri, 6)
    mesh.destroy()


@pytest.mark.parametrize("op,k", [(bem.LAPLACE_SLP, 0.0), (bem.LAPLACE_DLP, 0.0), (bem.LAPLACE_ADLP, 0.0),
                                  (bem.HELMHOLTZ_SLP, 4.0), (bem.HELMHOLTZ_DLP, 4.0)])
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (37, 150), (129, 3)])
def test_dp1_entries_vs_oracle(ico3, op, k, shape):
    xyz, tri, mesh, om = ico3
    n = 3 * tri.shape[0]
    rng = np.random.Generator(np.random.PCG64(31))
    rows = rng.choice(n, shape[0], replace=False).astype(np.int32)
    cols = rng.choice(n, shape[1], replace=False).astype(np.int32)
    ref = om.entries(op, O.DP1, k, rows, cols, near=O.NEAR_SKIP)
    g64 = bem.eval_entries(mesh, op, bem.DP1, k, rows, cols, prec=bem.FP64, near=bem.NEAR_SKIP)
    g32 = bem.eval_entries(mesh, op, bem.DP1, k, rows, cols, prec=bem.FP32, near=bem.NEAR_SKIP)
    scale = np.abs(ref).max()
    if scale == 0.0:
        assert not g64.any() and not g32.any()
        return
    assert np.abs(g64 - ref).max() <= 1e-11 * scale
    if op == bem.LAPLACE_SLP:
        nz = ref != 0
        assert np.all(g32[~nz] == 0)
        assert np.max(np.abs(g32[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-5
    else:
        bound = 1e-4 if bem.is_complex(op) else 1e-5
        assert np.abs(g32.astype(ref.dtype) - ref).max() <= bound * scale


@pytest.mark.parametrize("op", [bem.LAPLACE_SLP, bem.LAPLACE_DLP])
def test_dp1_singular_pairs_vs_oracle_local_matrices(op):
    xyz, tri = inputs.icosphere(2)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    nt = tri.shape[0]
    rows = np.arange(0, 3 * nt, 17, dtype=np.int32)
    cols = np.arange(3 * nt, dtype=np.int32)
    got = bem.eval_entries(mesh, op, bem.DP1, 0.0, rows, cols, prec=bem.FP64, near=bem.NEAR_SINGULAR)
    skip = bem.eval_entries(mesh, op, bem.DP1, 0.0, rows, cols, prec=bem.FP64, near=bem.NEAR_SKIP)
    pairs = [(r // 3, c // 3) for r in rows for c in cols if set(tri[r // 3]) & set(tri[c // 3])]
    near = np.array([[bool(set(tri[r // 3]) & set(tri[c // 3])) for c in cols] for r in rows])
    assert np.array_equal(got[~near], skip[~near])
    uniq = sorted(set(pairs))
    idx = {p: i for i, p in enumerate(uniq)}
    L = (4 * om.nearfield_p1_local(op, [p[0] for p in uniq], [p[1] for p in uniq], 5) -
         om.nearfield_p1_local(op, [p[0] for p in uniq], [p[1] for p in uniq], 4)) / 3
    ref = np.zeros_like(got)
    for i, r in enumerate(rows):
        for j, c in enumerate(cols):
            if near[i, j]:
                ref[i, j] = L[idx[(r // 3, c // 3)], r % 3, c % 3]
    err = np.abs((got - skip) - ref)[near].max() / np.abs(ref).max()
    print(f"DP1 op {op}: {near.sum()} singular entries, max rel err {err:.2e}")
    assert err <= 1e-6
    mesh.destroy()


@pytest.mark.parametrize("op,k", [(bem.LAPLACE_HYPS, 0.0), (bem.HELMHOLTZ_HYPS, 2.0)])
@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_hyps_via_slp_matvec_vs_direct_oracle(ico3, op, k, prec):
    xyz, tri, mesh, om = ico3
    nv = xyz.shape[0]
    H = bem.hmat_assemble(mesh, op, bem.P1, k, leaf_size=48, eta=1.0, aca_tol=1e-6, max_rank=150, n_workers=4,
                          blocks_per_worker=16, prec=prec, dense_mode=1, hyps_via_slp=1)
    idx = np.arange(nv, dtype=np.int32)
    A = om.entries(op, O.P1, k, idx, idx, near=O.NEAR_SKIP)
    rng = np.random.Generator(np.random.PCG64(5))
    worst = 0.0
    for x in (xyz[:, 0].copy(), rng.normal(size=nv)):
        if bem.is_complex(op):
            x = x + 0.5j * x[::-1]
        y = H.matvec(x)
        err = np.linalg.norm(y - A @ x) / np.linalg.norm(A @ x)
        worst = max(worst, err)
    st = H.stats()
    print(f"op {op} prec {prec}: matvec rel err {worst:.2e}, DP1 blocks {st['admissible_blocks']}, "
          f"mean rank {st['rank_sum'] / max(1, st['admissible_blocks']):.2f}")
    assert worst <= 1e-5
    H.destroy()


def test_hyps_via_slp_complete_sphere_eigenvalue():
    xyz, tri = inputs.icosphere(3)
    nv, nt = xyz.shape[0], tri.shape[0]
    mesh = bem.mesh_create(xyz, tri, 6)
    H = bem.hmat_assemble(mesh, bem.LAPLACE_HYPS, bem.P1, 0.0, leaf_size=48, eta=1.0, aca_tol=1e-8, max_rank=150,
                          n_workers=4, blocks_per_worker=8, prec=bem.FP64, dense_mode=2, hyps_via_slp=1)
    D = bem.hmat_assemble(mesh, bem.LAPLACE_HYPS, bem.P1, 0.0, leaf_size=32, eta=1.0, aca_tol=1e-8, max_rank=100,
                          n_workers=4, blocks_per_worker=8, prec=bem.FP64, dense_mode=2)
    u = xyz[:, 0].copy()
    Du = H.matvec(u)
    area = 0.5 * np.linalg.norm(np.cross(xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 0]]), axis=1)
    Mu = np.zeros(nv)
    for t in range(nt):
        Mu[tri[t]] += area[t] / 12.0 * (np.ones((3, 3)) + np.eye(3)) @ u[tri[t]]
    eig = np.linalg.norm(Du - (2.0 / 3.0) * Mu) / np.linalg.norm((2.0 / 3.0) * Mu)
    rel = np.linalg.norm(Du - D.matvec(u)) / np.linalg.norm(Du)
    print(f"via-SLP complete: eigenvalue residual {eig:.2e}, against the direct complete H-matrix {rel:.2e}")
    assert eig <= 5e-3 and rel <= 1e-6
    H.destroy()
    D.destroy()
    mesh.destroy()


def test_hyps_via_slp_fp32_ranks_level6():
    xyz, tri = inputs.icosphere(6)
    mesh = bem.mesh_create(xyz, tri, 6)
    st = {}
    for prec in (bem.FP64, bem.FP32):
        H = bem.hmat_assemble(mesh, bem.LAPLACE_HYPS, bem.P1, 0.0, leaf_size=100, eta=1.0, aca_tol=1e-5,
                              max_rank=200, n_workers=10, blocks_per_worker=180, prec=prec, dense_mode=0,
                              hyps_via_slp=1)
        st[prec] = H.stats()
        H.destroy()
    r32, r64 = st[bem.FP32]["rank_sum"], st[bem.FP64]["rank_sum"]
    print(f"level 6 via SLP: rank sum FP32 {r32} FP64 {r64}, requests FP32 {st[bem.FP32]['aca_requests']} "
          f"FP64 {st[bem.FP64]['aca_requests']}, seconds {st[bem.FP32]['seconds']:.3f} / {st[bem.FP64]['seconds']:.3f}")
    assert r32 <= 1.2 * r64
    mesh.destroy()
