"""Dynamic weak constraints on the GPU: proximity detection against a brute
force reference, the incremental recolouring against the oracle's (bit
exact), and solves, residuals and backward-Euler steps with contacts
against the oracle run with the workspace's colouring.  Tolerances as for
the other parity tests: FP64 1e-10 relative, FP32 1e-5."""
import numpy as np
import pytest

import oracle as O
from paper_2306_09021_amd import scenarios as S

from .gpu_util import announce, dev_x, host, rel_err, require_gpu, torch, workspace
from .test_oracle_contacts import add_contacts, brute_contacts
from .test_oracle_solve import check_valid_coloring

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def near_blocks(n=5, gap=0.05, shift=0.04, model="corotated"):
    sc = S.two_blocks(n, gap=gap, model=model, drive=0.02)
    x = sc.initial_iterate()
    half = sc.n_verts // 2
    x[half:, 0] -= shift                       # the right block moved toward the left one
    x[sc.dirichlet_idx] = sc.dirichlet_x
    return sc, x


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_detection_matches_brute_force(real):
    sc, x = near_blocks()
    xr = x.astype(np.float32).astype(np.float64) if real == "f32" else x
    op = O.make_problem(sc)
    ref_p, ref_n = brute_contacts(xr, sc.tets, op.is_dir, 0.05)
    announce("contact detection %s" % real)
    ws = workspace([sc], real)
    pairs, normals = ws.detect_contacts(dev_x(xr, real), 0.05, max_pairs=4096)
    assert ref_p.shape[0] > 10
    assert np.array_equal(host(pairs).astype(np.int64), ref_p.astype(np.int64))
    assert np.abs(host(normals) - ref_n).max() <= 1e-12


def test_recolouring_matches_oracle():
    sc, x = near_blocks()
    op = O.make_problem(sc)
    pairs, normals = brute_contacts(x, sc.tets, op.is_dir, 0.05)
    col0, _ = O.color(op)
    op2 = O.make_problem(add_contacts(sc, pairs, normals, 1e3))
    nodes = np.unique(pairs.reshape(-1))
    nodes = nodes[op2.is_dir[nodes] == 0]
    ref, _ = O.recolor(op2, col0, nodes)
    announce("recolouring after contacts")
    ws = workspace([sc], "f64")
    assert np.array_equal(ws.colors(), col0)
    ws.set_contacts(torch.tensor(pairs, dtype=torch.int32, device="cuda"),
                    torch.tensor(normals, dtype=torch.float64, device="cuda"), 1e3)
    got = ws.colors()
    assert np.array_equal(got, ref)
    check_valid_coloring(op2, got)
    assert np.any(got != col0)          # the contacts forced some vertex to move


@pytest.mark.parametrize("real,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_quasistatic_solve_with_contacts(real, tol):
    sc, x = near_blocks(model="nh")
    op = O.make_problem(sc)
    pairs, normals = brute_contacts(x, sc.tets, op.is_dir, 0.05)
    sc2 = add_contacts(sc, pairs, normals, 1e3)
    announce("solve with contacts %s" % real)
    ws = workspace([sc], real)
    ws.set_contacts(torch.tensor(pairs, dtype=torch.int32, device="cuda"),
                    torch.tensor(normals, dtype=torch.float64, device="cuda"), 1e3)
    col = ws.colors()
    op2 = O.make_problem(sc2)
    kw = dict(accel="chebyshev", rho=0.9, gamma=1.3, safeguard="backtrack")
    xo, sto = O.solve(op2, col, x, max_sweeps=40, **kw)
    xg = dev_x(x, real)
    ws.solve(xg, max_sweeps=40, rel_tol=0.0, check_every=40, **kw)
    assert rel_err(host(xg), xo) <= tol
    # FP64 residual and energy include the contact terms
    if real == "f64":
        n_o, E_o, r_o = O.residual(op2, xo)
        rn, E, r = ws.residual(xg, want_r=True)
        assert abs(rn[0] - n_o) <= 1e-9 * n_o
        assert abs(E[0] - E_o) <= 1e-9 * abs(E_o)


def test_backward_euler_steps_with_detection():
    """The paper's collision loop: every step detects contacts at the
    current positions, installs them (stiffness 1e8, anisotropic along the
    pair's normal) and takes a backward-Euler step (dt = 0.002); FP64
    against the oracle with the same contacts and colouring."""
    sc = S.two_blocks(5, gap=0.02, model="corotated", drive=0.06)
    op = O.make_problem(sc)
    ws = workspace([sc], "f64")
    dt, kn, radius = 0.002, 1e8, 0.03
    x_prev = sc.initial_iterate()
    x_n = x_prev.copy()
    announce("backward Euler with detection, 5 steps")
    n_contacts = []
    for step in range(5):
        xg = dev_x(x_n, "f64")
        pairs, normals = ws.detect_contacts(xg, radius, max_pairs=4096)
        p_h, n_h = host(pairs).astype(np.int64), host(normals)
        ref_p, ref_n = brute_contacts(x_n, sc.tets, op.is_dir, radius)
        assert np.array_equal(p_h, ref_p.astype(np.int64))
        n_contacts.append(p_h.shape[0])
        ws.set_contacts(pairs, normals, kn)
        ws.set_inertia(dt, torch.tensor(x_n, device="cuda"), torch.tensor(x_prev, device="cuda"))
        ws.solve(xg, max_sweeps=30, rel_tol=0.0, check_every=30, accel="none",
                 safeguard="backtrack")
        op2 = O.make_problem(add_contacts(sc, ref_p, ref_n, kn))
        op2.set_inertia(dt, x_n, x_prev)
        xo, _ = O.solve(op2, ws.colors(), x_n, max_sweeps=30, accel="none", safeguard="backtrack")
        assert rel_err(host(xg), xo) <= 1e-10, step
        x_prev, x_n = x_n, xo
    assert max(n_contacts) > 0


def test_detection_overflow_is_reported_and_recoverable():
    """More pairs than max_pairs: the call fails with PBNG_EINVAL (nothing is
    written past max_pairs), and a following call with room, which grows the
    scratch, returns the full sorted set."""
    from paper_2306_09021_amd import pbng
    sc, x = near_blocks()
    op = O.make_problem(sc)
    ref_p, _ = brute_contacts(x, sc.tets, op.is_dir, 0.05)
    assert ref_p.shape[0] > 8
    announce("contact detection overflow then growth")
    ws = workspace([sc], "f64")
    with pytest.raises(pbng.PBNGError) as e:
        ws.detect_contacts(dev_x(x, "f64"), 0.05, max_pairs=4)
    assert e.value.code == -1
    pairs, _ = ws.detect_contacts(dev_x(x, "f64"), 0.05, max_pairs=8192)
    assert np.array_equal(host(pairs).astype(np.int64), ref_p.astype(np.int64))


def test_colliding_blocks_full_size_substep():
    """The benchmark's collision workload at its size (two 16^3 corotated
    blocks, 8192 vertices, 33,750 tets, PBNG_MIXED): with the right block
    pushed into contact range, detection against brute force, the
    recolouring against the oracle's, then one substep (dt = 1/510 s,
    k_n = 1e8, 8 Chebyshev iterations, no safeguard) against the oracle run
    with the same contacts, colouring and inertia."""
    sc = S.two_blocks(16, gap=0.02, model="corotated", drive=0.0)
    x = sc.initial_iterate()
    half = sc.n_verts // 2
    x[half:, 0] -= 0.03
    x[sc.dirichlet_idx] = sc.dirichlet_x
    op = O.make_problem(sc)
    radius, kn, dt = 0.03, 1e8, 1.0 / 30.0 / 17.0
    ref_p, ref_n = brute_contacts(x, sc.tets, op.is_dir, radius)
    assert ref_p.shape[0] > 50
    announce("colliding blocks 2 x 16^3 one substep mixed")
    ws = workspace([sc], "mixed")
    xg = dev_x(x, "mixed")
    pairs, normals = ws.detect_contacts(xg, radius, max_pairs=1 << 16)
    assert np.array_equal(host(pairs).astype(np.int64), ref_p.astype(np.int64))
    assert np.abs(host(normals) - ref_n).max() <= 1e-12
    col0 = ws.colors()
    ws.set_contacts(pairs, normals, kn)
    op2 = O.make_problem(add_contacts(sc, ref_p, ref_n, kn))
    nodes = np.unique(ref_p.reshape(-1))
    nodes = nodes[op2.is_dir[nodes] == 0]
    ref_col, _ = O.recolor(op2, col0, nodes)
    assert np.array_equal(ws.colors(), ref_col)
    x_prev = x - 1e-4
    x_prev[sc.dirichlet_idx] = sc.dirichlet_x
    ws.set_inertia(dt, torch.tensor(x, device="cuda"), torch.tensor(x_prev, device="cuda"))
    kw = dict(accel="chebyshev", rho=0.95, gamma=1.2, safeguard="none")
    ws.solve(xg, max_sweeps=8, rel_tol=0.0, check_every=8, **kw)
    op2.set_inertia(dt, x, x_prev)
    xo, _ = O.solve(op2, ws.colors(), x, max_sweeps=8, **kw)
    assert rel_err(host(xg), xo) <= 1e-5


def test_removing_contacts_keeps_recoloured_phases():
    """Contacts installed (some vertices recoloured) and then removed: the
    recoloured vertices keep their new colours, so every later solve and
    adjoint still runs their phases from the vertex lists, also with no
    other weak constraint, plane, inertia or second instance.  FP64 against
    the oracle with the workspace's colouring and no contacts."""
    from oracle import dense as D
    from paper_2306_09021_amd import pbng
    sc, x = near_blocks(model="nh")
    op = O.make_problem(sc)
    pairs, normals = brute_contacts(x, sc.tets, op.is_dir, 0.05)
    announce("contacts installed then removed, solve and adjoint f64")
    ws = workspace([sc], "f64")
    col0 = ws.colors()
    ws.set_contacts(torch.tensor(pairs, dtype=torch.int32, device="cuda"),
                    torch.tensor(normals, dtype=torch.float64, device="cuda"), 1e3)
    ws.set_contacts(None, None, 1e3)
    col = ws.colors()
    assert np.any(col != col0)
    check_valid_coloring(op, col)
    kw = dict(accel="chebyshev", rho=0.9, gamma=1.3, safeguard="backtrack")
    xo, _ = O.solve(op, col, x, max_sweeps=40, **kw)
    xg = dev_x(x, "f64")
    ws.solve(xg, max_sweeps=40, rel_tol=0.0, check_every=40, **kw)
    assert rel_err(host(xg), xo) <= 1e-10
    # adjoint at an equilibrium, against a dense solve
    xe, _ = O.solve(op, col, x, max_sweeps=20000, rel_tol=1e-13, check_every=50, **kw)
    g = 2.0 * (xe - sc.rest_pos) * (op.is_dir == 0)[:, None]
    lam_d = D.adjoint_dense(op, xe, g)
    o = pbng.adjoint_opts(rel_tol=1e-12, max_sweeps=20000, check_every=20, accel="chebyshev", rho=0.9,
                          gamma=1.0)
    rc, out, st = ws.adjoint(dev_x(xe, "f64"), dev_x(g, "f64"), o, want=("lam_vec",))
    lv = host(out["lam_vec"])
    assert np.linalg.norm(lv - lam_d) / np.linalg.norm(lam_d) <= 1e-8


def test_state_changes_in_sequence_with_graph_replay():
    """One workspace through every state change, with graph replay on
    (sweeps_per_graph = 4 on a non-null stream): quasistatic solve, inertia
    on, contacts in (recolouring), new materials, contacts out, inertia off,
    new Dirichlet targets.  After each change a 24-sweep solve in FP64
    against the oracle set up in the same state (1e-10)."""
    import copy
    sc = S.two_blocks(5, gap=0.02, model="corotated", drive=0.0)
    half = sc.n_verts // 2
    x = sc.initial_iterate()
    x[half:, 0] -= 0.04
    x[sc.dirichlet_idx] = sc.dirichlet_x
    radius, kn, dt = 0.05, 1e4, 0.01
    kw = dict(accel="chebyshev", rho=0.9, gamma=1.2, safeguard="backtrack")
    stream = torch.cuda.Stream()
    announce("state changes in sequence with graph replay f64")
    with torch.cuda.stream(stream):
        ws = workspace([sc], "f64")
        state = dict(sc=copy.copy(sc), contacts=None, inertia=None, mu=None, lam=None)

        def check(tag, x_start):
            xg = dev_x(x_start, "f64")
            ws.solve(xg, max_sweeps=24, rel_tol=0.0, check_every=24, sweeps_per_graph=4, stream=stream, **kw)
            stream.synchronize()
            s = state["sc"] if state["contacts"] is None else add_contacts(state["sc"], *state["contacts"], kn)
            op = O.make_problem(s, mu=state["mu"], lam=state["lam"])
            if state["inertia"] is not None:
                op.set_inertia(dt, *state["inertia"])
            xo, _ = O.solve(op, ws.colors(), x_start, max_sweeps=24, **kw)
            e = rel_err(host(xg), xo)
            print(tag, "rel err", e)
            assert e <= 1e-10, tag
            return host(xg)

        x1 = check("quasistatic", x)
        x_prev = x - 1e-3
        x_prev[sc.dirichlet_idx] = sc.dirichlet_x
        ws.set_inertia(dt, torch.tensor(x, device="cuda"), torch.tensor(x_prev, device="cuda"), stream=stream)
        state["inertia"] = (x, x_prev)
        check("inertia on", x)
        pairs, normals = ws.detect_contacts(dev_x(x, "f64"), radius, max_pairs=4096, stream=stream)
        assert pairs.shape[0] > 0
        ws.set_contacts(pairs, normals, kn, stream=stream)
        state["contacts"] = (host(pairs).astype(np.int64), host(normals))
        check("contacts in", x)
        from paper_2306_09021_amd import pbng
        mu0, lam0 = pbng.lame(sc.E, sc.nu)
        nt = sc.n_tets
        mu = np.full(nt, float(mu0)) * np.linspace(0.5, 1.5, nt)
        lam = np.full(nt, float(lam0)) * np.linspace(1.5, 0.5, nt)
        ws.set_materials(torch.tensor(mu, device="cuda"), torch.tensor(lam, device="cuda"), stream=stream)
        state["mu"], state["lam"] = mu, lam
        check("new materials", x)
        ws.set_contacts(None, None, kn, stream=stream)
        state["contacts"] = None
        check("contacts out", x)
        ws.set_inertia(0.0, stream=stream)
        state["inertia"] = None
        check("inertia off", x1)
        xd = sc.dirichlet_x.copy()
        xd[:, 1] += 0.05
        ws.set_dirichlet(torch.tensor(xd, device="cuda"), stream=stream)
        s2 = copy.copy(sc)
        s2.dirichlet_x = xd
        state["sc"] = s2
        x2 = x1.copy()
        x2[sc.dirichlet_idx] = xd
        check("new Dirichlet targets", x2)


def test_batched_instances_with_contacts():
    """Two instances (two-block scenes pushed together by different amounts)
    in one workspace: detection keeps pairs inside each instance, contacts
    and recolouring act per instance, and each instance's solve equals its
    own oracle solve with its contacts and the workspace's colouring (FP64)."""
    scs, xs = [], []
    for k, shift in enumerate((0.035, 0.045)):
        sc = S.two_blocks(5, gap=0.02, model="nh", drive=0.0)
        x = sc.initial_iterate()
        x[sc.n_verts // 2:, 0] -= shift
        x[sc.dirichlet_idx] = sc.dirichlet_x
        scs.append(sc)
        xs.append(x)
    off = np.cumsum([0] + [s.n_verts for s in scs])
    xall = np.concatenate(xs)
    announce("batched instances with contacts f64")
    ws = workspace(scs, "f64")
    radius, kn = 0.05, 1e4
    pairs, normals = ws.detect_contacts(dev_x(xall, "f64"), radius, max_pairs=8192)
    p_h, n_h = host(pairs).astype(np.int64), host(normals)
    ws.set_contacts(pairs, normals, kn)
    kw = dict(accel="chebyshev", rho=0.9, gamma=1.2, safeguard="backtrack")
    xg = dev_x(xall, "f64")
    ws.solve(xg, max_sweeps=30, rel_tol=0.0, check_every=30, **kw)
    xg, col = host(xg), ws.colors()
    counts = []
    for q, sc in enumerate(scs):
        inq = (p_h[:, 0] >= off[q]) & (p_h[:, 0] < off[q + 1])
        assert np.all((p_h[inq, 1] >= off[q]) & (p_h[inq, 1] < off[q + 1]))
        op = O.make_problem(sc)
        ref_p, ref_n = brute_contacts(xs[q], sc.tets, op.is_dir, radius)
        assert np.array_equal(p_h[inq] - off[q], ref_p.astype(np.int64))
        counts.append(int(inq.sum()))
        op2 = O.make_problem(add_contacts(sc, ref_p, ref_n, kn))
        cq = col[off[q]:off[q + 1]]
        check_valid_coloring(op2, cq)
        xo, _ = O.solve(op2, cq, xs[q], max_sweeps=30, **kw)
        assert rel_err(xg[off[q]:off[q + 1]], xo) <= 1e-10, q
    assert counts[0] > 0 and counts[1] > 0
