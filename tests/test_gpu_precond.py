"""Block-Jacobi preconditioner, batched BSR values and GMRES iteration counts
against the CPU oracle, through the C ABI.

With right preconditioning x = M^{-1} V y undoes the M^{-1} of A M^{-1}, so a
wrong (but non-singular) inverse would still give correct solutions: the
inverse and A M^{-1} are therefore compared with the oracle's diagonal blocks
directly.  The reference inverse is LAPACK's (numpy) of the oracle's FP64
diagonal blocks, which shares nothing with either side's Gauss-Jordan."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_02941_amd import workloads as W

from tests import dgcases as DC

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_02941_amd import api as A
    A.lib()
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_precond(M, B, row_ptr, col_idx):
    """(D^{-1} [T, n, n], A_KL D_L^{-1} for the off-diagonal blocks in BSR order)
    from the oracle's blocks; LAPACK inverses."""
    dinv = np.linalg.inv(B.diag)
    n = B.diag.shape[1]
    T = M.T
    a = M.int_el[:, 0].astype(np.int64)
    b = M.int_el[:, 1].astype(np.int64)
    keys = np.concatenate([a * T + b, b * T + a])
    blocks = np.concatenate([B.off_ij, B.off_ji])
    order = np.argsort(keys)
    keys, blocks = keys[order], blocks[order]
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    rows = np.repeat(np.arange(T), np.diff(row_ptr))
    off = np.ones(len(col_idx), dtype=bool)
    off[row_ptr[:-1]] = False  # the diagonal block leads each block row
    K, L = rows[off], col_idx[off]
    pos = np.searchsorted(keys, K * T + L)
    assert np.all(keys[np.minimum(pos, len(keys) - 1)] == K * T + L), "BSR pattern differs from the oracle's edges"
    if len(K) == 0:
        return dinv, np.zeros((0, n, n))
    return dinv, blocks[pos] @ dinv[L]


def blockwise(gpu, ref):
    """(normwise relative error, largest per-block relative error, worst block index)."""
    d = np.linalg.norm((gpu - ref).reshape(len(ref), -1), axis=1)
    r = np.linalg.norm(ref.reshape(len(ref), -1), axis=1)
    per = d / np.maximum(r, 1e-300)
    return float(np.linalg.norm(d) / max(np.linalg.norm(r), 1e-300)), float(per.max()), int(per.argmax())


def check_precond(dinv_g, ahat_g, dinv_o, ahat_o, diag_blocks, mixed, label):
    """FP64 inverse within 1e-12 (normwise and per block, the per-block bound
    scaled by the block's condition number above 1e2: a backward-stable
    inverse errs by about cond * 1e-16); A D^{-1} the same in FP64, within
    FP32 rounding (2^-23 scaled by sqrt(n)) when mixed."""
    cond = np.linalg.cond(diag_blocks)
    nw, pb, w = blockwise(dinv_g, dinv_o)
    scaled = np.linalg.norm((dinv_g - dinv_o).reshape(len(dinv_o), -1), axis=1) / \
        np.linalg.norm(dinv_o.reshape(len(dinv_o), -1), axis=1) / np.maximum(1.0, cond / 1e2)
    _say("  %s: D^-1 normwise %.2e, worst block %.2e (block %d, cond %.1e), cond-scaled %.2e"
         % (label, nw, pb, w, cond[w], scaled.max()))
    assert nw <= 1e-12, (label, nw)
    assert scaled.max() <= 1e-12, (label, scaled.max())
    if len(ahat_o):
        nw2, pb2, w2 = blockwise(ahat_g, ahat_o)
        _say("  %s: A D^-1 normwise %.2e, worst block %.2e" % (label, nw2, pb2))
        n = ahat_o.shape[1]
        bound = 2.0 ** -23 * np.sqrt(n) * 4 if mixed else 1e-12
        assert nw2 <= bound, (label, nw2)
        if not mixed:
            assert pb2 <= 1e-12 * max(1.0, float(cond.max()) / 1e2), (label, pb2)


SOLVER_CASES = ["c1_8x8_p1_sipg", "jit13_p1_m3_mixedbc_rot", "jit11_p2_m1_mixedbc_const", "jit11_p3_m2_mixedbc_const",
                "jit13_p4_m2_mixedbc_rot", "c2like_32_p2_m2", "c3like_24_p3_iipg", "c4like_20_p2_gauss",
                "jit11_p0_m1_mixedbc_const"]


def _case(name):
    for c in DC.small_cases():
        if c.name == name:
            return c
    raise KeyError(name)


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("name", SOLVER_CASES)
def test_solver_block_jacobi_matches_oracle(api, name, mixed):
    c = _case(name)
    _say("case %s (k = %d), mixed = %s" % (c.name, c.k, mixed))
    M, B = DC.oracle_system(c)
    mesh = api.Mesh.from_arrays(c.mesh, c.k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(c, mesh, api))
    s = api.Solver(mesh, restart=64, rel_tol=1e-10, mixed=mixed)
    s.setup(vals)
    dinv, ahat = s.preconditioner()
    rp, ci = mesh.structure()
    torch.cuda.synchronize()
    dinv_o, ahat_o = oracle_precond(M, B, rp.cpu().numpy(), ci.cpu().numpy())
    check_precond(dinv.cpu().numpy(), ahat.double().cpu().numpy(), dinv_o, ahat_o, B.diag, mixed, c.name)


@pytest.mark.parametrize("name,restart,tol", [("c1_8x8_p1_sipg", 32, 1e-12), ("c2like_32_p2_m2", 128, 1e-10),
                                              ("c2like_32_p2_m1", 128, 1e-10), ("c4like_20_p2_gauss", 40, 1e-10),
                                              ("jit13_p2_m3_mixedbc_rot", 50, 1e-10)])
def test_fp64_iteration_counts_match_oracle_gmres(api, name, restart, tol):
    """One Arnoldi vector per Gram-Schmidt pass, FP64: the GPU's iteration
    count equals the oracle's GMRES (same restart, same right block-Jacobi,
    same stopping test) within a few steps (the oracle orthogonalises by
    modified, the GPU by classical Gram-Schmidt)."""
    c = _case(name)
    M, B = DC.oracle_system(c)
    _, its_o, rel_o, conv = O.gmres(B, restart=restart, tol=tol)
    assert conv
    mesh = api.Mesh.from_arrays(c.mesh, c.k)
    vals, rhs = api.assemble(mesh, DC.gpu_problem(c, mesh, api))
    A = B.to_scipy()
    for pers in (False, "auto"):
        s = api.Solver(mesh, restart=restart, rel_tol=tol, max_iters=20000, block=1, persistent=pers)
        s.setup(vals)
        x = torch.zeros_like(rhs)
        rep = s.solve(rhs, x)
        rr = float(np.linalg.norm(B.rhs - A @ x.cpu().numpy()) / np.linalg.norm(B.rhs))
        _say("  %s restart %d persistent=%s: GPU %d its (LDS path %d), oracle %d its; oracle-judged %.2e"
             % (name, restart, pers, rep.iters, rep.persistent, its_o, rr))
        assert rep.converged and rr <= 1.01 * tol
        assert abs(rep.iters - its_o) <= 3 + its_o // 50, (name, pers, rep.iters, its_o)


def _c4_slice():
    """Every 128th instance of the seeded 4096-instance batched workload (full
    sizes, N up to 128), plus its two smallest instances."""
    insts = W.sample_instances(4096, seed=0)
    idx = sorted(set(range(0, 4096, 128)) | set(np.argsort([i.N for i in insts])[:2].tolist()))
    return [insts[i] for i in idx], idx


def _oracle_instance(inst):
    m = W.structured_mesh(inst.N)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    sigma, kappa = O.default_penalty(O.SIPG, inst.k)
    B = O.assemble(M, inst.k, sigma=sigma, kappa=kappa, eps=inst.eps, bx=inst.b[0], by=inst.b[1],
                   alpha=inst.alpha, f=O.Field.gauss_sum([tuple(t) for t in inst.gauss]), gD=0.0)
    return m, M, B


@pytest.mark.parametrize("mixed", [True, False])
def test_batched_values_and_preconditioner_match_oracle(api, mixed):
    """A slice of the batched workload: the FP64 BSR values and load vector of
    every instance blockwise at 1e-12, and its block-Jacobi preconditioner, on
    both solve paths (small instances persistent, the rest lockstep)."""
    insts, idx = _c4_slice()
    split = 8000
    _say("C4 slice: %d instances (workload indices %s), lockstep from %d dofs, mixed=%s"
         % (len(insts), idx, split, mixed))
    b = api.Batch([(W.structured_mesh(i.N), api.instance_problem(i)) for i in insts], mixed=mixed, rel_tol=1e-10,
                  inner_tol=1e-5, block_threads=256, lockstep_min_dofs=split, log=_say)
    x, rep = b.alloc()
    b.run(x, rep)
    torch.cuda.synchronize()
    R = b.reports(rep)
    paths = set()
    for i, inst in enumerate(insts):
        assert R[i]["status"] == 0 and R[i]["rel_res"] <= 1e-10, (i, R[i])
        m, M, B = _oracle_instance(inst)
        n = (inst.k + 1) * (inst.k + 2) // 2
        mesh = api.Mesh.from_arrays(m, inst.k)
        rp, ci = mesh.structure()
        vals, rhs = b.system(i, n, mesh.nnzb)
        dinv, ahat = b.preconditioner(i, n, mesh.nnzb)
        torch.cuda.synchronize()
        Ag = api.bsr_to_scipy(mesh, vals, rp, ci)
        A = B.to_scipy()
        err = DC.rel_fro(Ag, A)
        mx, scale = DC.max_abs_diff(Ag, A)
        ferr = DC.rel_fro(rhs.cpu().numpy(), B.rhs)
        path = "lockstep" if b.offsets[i + 1] - b.offsets[i] >= split else "persistent"
        paths.add(path)
        _say("  instance %d (k %d, N %d, eps %.1e, %s): values %.2e (max %.2e of %.2e), rhs %.2e"
             % (idx[i], inst.k, inst.N, inst.eps, path, err, mx, scale, ferr))
        assert err <= 1e-12 and mx <= 1e-12 * scale and ferr <= 1e-12
        dinv_o, ahat_o = oracle_precond(M, B, rp.cpu().numpy(), ci.cpu().numpy())
        check_precond(dinv.cpu().numpy(), ahat.double().cpu().numpy(), dinv_o, ahat_o, B.diag, mixed,
                      "instance %d %s" % (idx[i], path))
        rr = float(np.linalg.norm(B.rhs - A @ b.segment(x, i).cpu().numpy()) / np.linalg.norm(B.rhs))
        assert rr <= 1.01e-10, (idx[i], rr)
    assert paths == {"lockstep", "persistent"}
