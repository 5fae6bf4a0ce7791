"""Batched launch shapes (a9): every chunk size and graph replay of the
batched Krylov chunks gives each scene's adjoint within the oracle's 1e-9
bar, graph replay is bitwise equal to direct launches of the same chunks,
and the batched autotuner returns a member of the supported set."""

import numpy as np
import pytest

from gpu_helpers import contact_tensors, rel, torch_cuda
from oracle import adjoint as adj
from test_gpu_batch import _cases

pytestmark = pytest.mark.gpu


def _batch():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    cases = _cases()
    spec0 = cases[0][0]
    batch = native.Batch([(c[0].mesh.rest, c[0].mesh.tets, c[0].E, c[0].nu) for c in cases], spec0.density,
                         spec0.h, spec0.eps, spec0.gravity, spec0.planes, spec0.contact_margin,
                         [max(1, c[3].contacts.n) for c in cases])
    keep, states = [], []
    for c in cases:
        tens = contact_tensors(c[3])
        keep.append(tens)
        states.append(native.make_contact_state(c[3].contacts.n, tens["vid"], tens["fric"], tens["frame"],
                                                tens["delta"], tens["lam"], c[3].mu))
    dev = "cuda"
    q = torch.tensor(np.concatenate([c[2] for c in cases]), device=dev)
    gq = torch.tensor(np.concatenate([c[4] for c in cases]), device=dev)
    gv = torch.tensor(np.concatenate([c[5] for c in cases]), device=dev)
    return batch, keep, states, q, gq, gv


def test_batched_chunks_and_graphs_agree_with_oracle():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    cases = _cases()
    refs = [adj.adjoint_step(c[1], c[2], c[3], c[4], c[5], c[0].eps, c[0].E, c[0].nu).z for c in cases]
    batch, keep, states, q, gq, gv = _batch()
    opts = native.solve_opts(rtol=1e-12, maxit=3000, restart=64)
    zs = {}
    for chunk, graph, a_inv in ((8, 0, 0), (8, 1, 0), (2, 0, 0), (4, 1, 0), (16, 1, 0), (8, 0, 2), (8, 1, 2),
                                (4, 0, 1)):
        native.batch_set_tuning(batch, chunk=chunk, graph=graph, a_inv=a_inv)
        assert native.batch_get_tuning(batch) == {"chunk": chunk, "graph": graph, "a_inv": a_inv}
        native.batch_setup(batch, states, q, opts)
        for rep in range(2):  # graph mode: capture on the first solve, replay after
            z = torch.zeros_like(q)
            infos = native.batch_solve(batch, gq, gv, z, opts, raise_noconv=False)
            zn = z.cpu().numpy()
            errs = [rel(zn[batch.voff[k]:batch.voff[k + 1]], refs[k]) for k in range(len(cases))]
            print(f"chunk {chunk} graph {graph} a_inv {a_inv} rep {rep}: iters {[i.iters for i in infos]}, "
                  f"z err {max(errs):.2e}", flush=True)
            assert max(errs) <= 1e-9
            zs.setdefault((chunk, graph, a_inv), zn)
            assert np.array_equal(zs[(chunk, graph, a_inv)], zn)  # replay is deterministic
    assert np.array_equal(zs[(8, 0, 0)], zs[(8, 1, 0)])  # graph replay = direct launches of the same chunks
    assert np.array_equal(zs[(8, 0, 2)], zs[(8, 1, 2)])
    batch.close()


def test_batched_autotune_returns_supported_shape():
    torch = torch_cuda()
    from paper_2603_16478_amd import native
    batch, keep, states, q, gq, gv = _batch()
    opts = native.solve_opts(rtol=1e-8, maxit=3000, restart=64)
    native.batch_setup(batch, states, q, opts)
    z = torch.zeros_like(q)
    best = native.batch_autotune(batch, gq, gv, z, opts, reps=2)
    print("batched autotune", best, flush=True)
    assert best["chunk"] in (2, 4, 8, 16, 32) and best["graph"] in (0, 1) and best["a_inv"] in (0, 1, 2)
    assert native.batch_get_tuning(batch) == best
    with pytest.raises(native.AdjError):
        native.batch_set_tuning(batch, chunk=0)
    with pytest.raises(native.AdjError):
        native.batch_set_tuning(batch, chunk=8, graph=2)
    with pytest.raises(native.AdjError):
        native.batch_set_tuning(batch, chunk=8, graph=0, a_inv=3)
    batch.close()
