"""GPU: batched lockstep solves against solves alone (through the C ABI).

The batch runs each problem's PCG iterations with the same kernel bodies,
arguments and reduction orders as msp_solve on the same handle, so every
result must be bitwise the one the problem gets alone; the graph-captured
chunks (replayed several times per solve, with host synchronisation between
replays) must give the same bits again.  Parity with the oracle is the
single-problem tests' job; here one entry is also checked against a sparse
direct solve.
"""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _msp():
    import paper_2006_13387_amd as msp
    return msp


def _problems():
    # uneven sizes and both precisions: config-1 style fields on small
    # meshes, the 64x32 cantilever and a ragged mesh
    ps = [inputs.config(0),
          inputs.scaled_cantilever_2d((128, 64), 3001, precision=1),
          inputs.scaled_cantilever_2d((64, 32), 3002, sub=16, precision=0),
          inputs.scaled_cantilever_2d((96, 32), 3003, sub=16, precision=1)]
    return ps


def _solvers(ps):
    msp = _msp()
    out = []
    for p in ps:
        s = msp.Solver(p.desc, p.fixed)
        s.set_densities(torch.tensor(p.rho, device="cuda"))
        out.append(s)
    return out


def test_batch_matches_alone_bitwise_eager_and_graph():
    msp = _msp()
    ps = _problems()
    print(f"[batch] sizes {[p.desc['nel'] for p in ps]}", flush=True)
    alone = []
    solvers = _solvers(ps)
    fs = [torch.tensor(p.f, device="cuda") for p in ps]
    for s, f in zip(solvers, fs):
        u, info = s.solve(f, rtol=1e-8)
        print(f"[alone] status={info['status']} iters={info['iters']} "
              f"relres={info['relres_true']:.2e} restarts={info['restarts']}", flush=True)
        alone.append((u.clone(), info))
    b = msp.Batch()
    b.set_autotune(False)                  # the fixed shape: 16 iterations a chunk
    for use_graph in (False, True, True):
        us, infos = b.solve(solvers, fs, rtol=1e-8, use_graph=use_graph)
        torch.cuda.synchronize()
        for e, (u, info) in enumerate(zip(us, infos)):
            ua, ia = alone[e]
            assert torch.equal(u, ua), (use_graph, e)
            assert info["iters"] == ia["iters"], (use_graph, e)
            assert info["relres_true"] == ia["relres_true"]
            assert info["compliance"] == ia["compliance"]
            assert info["status"] == ia["status"]
    st = b.stats()
    print(f"[batch] stats {st}", flush=True)
    assert st["graph_chunks"] >= 2          # replays in two graph solves
    # one entry against the direct solve
    p = ps[1]
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    u = us[1].cpu().numpy()
    assert np.linalg.norm(u - ud) <= 1e-6 * np.linalg.norm(ud)
    b.close()
    for s in solvers:
        s.close()


def test_batch_warm_start_and_rejects_duplicates():
    msp = _msp()
    ps = [_problems()[k] for k in (0, 2)]   # two that reach 1e-8
    solvers = _solvers(ps)
    fs = [torch.tensor(p.f, device="cuda") for p in ps]
    b = msp.Batch()
    us, infos = b.solve(solvers, fs, rtol=1e-8)
    for i in infos:
        assert i["status"] == 0
    us2, infos2 = b.solve(solvers, fs, us=[u.clone() for u in us],
                          warm=[True, True], rtol=1e-8)
    for i in infos2:
        assert i["iters"] <= 1
        assert i["relres_true"] <= 1e-8
    with pytest.raises(msp.MspError):
        b.solve([solvers[0], solvers[0]], [fs[0], fs[0]])
    b.close()
    for s in solvers:
        s.close()


def test_batch_autotuner_changes_no_bits():
    """The launch-shape autotuner (iterations per chunk, first-level item
    order) measures its candidates on the first solves of a set of handles
    and then keeps the fastest: every solve, during and after the tuning,
    with and without graphs, gives the bits the problems get alone."""
    msp = _msp()
    ps = _problems()
    solvers = _solvers(ps)
    fs = [torch.tensor(p.f, device="cuda") for p in ps]
    alone = [s.solve(f, rtol=1e-8)[0].clone() for s, f in zip(solvers, fs)]
    b = msp.Batch()
    rounds = 0
    while not b.tuning()["tuned"] and rounds < 12:
        us, _ = b.solve(solvers, fs, rtol=1e-8, use_graph=True)
        for e, u in enumerate(us):
            assert torch.equal(u, alone[e]), (rounds, e)
        rounds += 1
    t = b.tuning()
    print(f"[batch] tuned after {rounds} solves: {t}", flush=True)
    assert t["tuned"]
    assert t["chunk"] in (8, 16, 32) and t["largest_first"] in (0, 1)
    assert all(c > 0 for c in t["cost_ms_per_iter_dof"])
    g0 = b.stats()["graph_chunks"]
    for _ in range(2):
        us, _ = b.solve(solvers, fs, rtol=1e-8, use_graph=True)
        for e, u in enumerate(us):
            assert torch.equal(u, alone[e]), e
    assert b.stats()["graph_chunks"] > g0      # the tuned shape is captured
    assert b.tuning()["chunk"] == t["chunk"]
    b.close()
    for s in solvers:
        s.close()
