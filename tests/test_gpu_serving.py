"""GPU tests of the continuous-batching server.

A request's field is bit-for-bit the same alone, in a mix of requests of
different sizes that overlap on the device, and through femh_solve with the
same options; cancellation and memory admission behave as documented."""
import time

import numpy as np
import pytest

import workloads as W
from paper_0704_2344_amd import femh as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = F.Context(0)
    yield c
    c.close()


def _requests(seed, count, n_hi=18):
    rng = np.random.default_rng(seed)
    return [W.serving_request(rng, n_lo=8, n_hi=n_hi, nrhs_hi=3) for _ in range(count)]


def _shape(prob, nrhs):
    return (nrhs, prob.nz + 1, prob.ny + 1, prob.nx + 1, 3)


def test_result_same_alone_and_in_mix(ctx):
    prob, waves = _requests(1, 1)[0]
    opts = dict(precision=F.FEMH_MIXED, rtol=1e-6)
    srv = F.Server(ctx, max_slots=8, chunk_iters=16)
    t = srv.submit(prob, waves, **opts)
    st, alone, stats = srv.poll(t, len(waves), _shape(prob, len(waves)))
    assert st == F.FEMH_OK, stats
    # the same request again, in the middle of a mix
    others = _requests(2, 6)
    tickets = [srv.submit(p, w, **opts) for p, w in others[:3]]
    t2 = srv.submit(prob, waves, **opts)
    tickets += [srv.submit(p, w, **opts) for p, w in others[3:]]
    st2, mixed, stats2 = srv.poll(t2, len(waves), _shape(prob, len(waves)))
    assert st2 == F.FEMH_OK
    np.testing.assert_array_equal(alone, mixed)
    for (p, w), tk in zip(others, tickets):
        s, _, _ = srv.poll(tk, len(w), _shape(p, len(w)))
        assert s == F.FEMH_OK
    rep = srv.report()
    assert rep["completed"] == 8 and rep["failed"] == 0
    assert rep["p99_seconds"] >= rep["p50_seconds"] > 0
    srv.close()
    # and the same through the plain solve path
    P = F.Problem(ctx, prob)
    H, s3, st3 = P.solve(waves, check_every=16, **opts)
    assert st3 == F.FEMH_OK
    np.testing.assert_array_equal(H, alone)
    P.close()


def test_cancel_and_admission(ctx):
    big, wbig = W.pec_sphere_batched(n=30, radius=0.8, nrhs=2, seed=9)
    small = _requests(3, 3, n_hi=12)
    srv = F.Server(ctx, max_slots=4, chunk_iters=16)
    tb = srv.submit(big, wbig, precision=F.FEMH_MIXED, rtol=1e-8)
    ts = [srv.submit(p, w, precision=F.FEMH_MIXED, rtol=1e-6) for p, w in small]
    assert srv.cancel(tb) == F.FEMH_OK
    st, _, _ = srv.poll(tb, 2, None, want_field=False)
    assert st == F.FEMH_E_CANCELLED
    for (p, w), t in zip(small, ts):
        s, _, _ = srv.poll(t, len(w), _shape(p, len(w)))
        assert s == F.FEMH_OK
    assert srv.cancel(123456) == F.FEMH_E_NOT_FOUND
    srv.close()
    # a budget that holds one small request at a time still serves them all,
    # and a request larger than the budget is refused at submission
    srv = F.Server(ctx, hbm_budget_bytes=64 << 20, max_slots=4)
    with pytest.raises(F.FemhError) as e:
        srv.submit(big, wbig)
    assert e.value.status == F.FEMH_E_OOM
    ts = [srv.submit(p, w, precision=F.FEMH_MIXED, rtol=1e-6) for p, w in small]
    for (p, w), t in zip(small, ts):
        s, _, _ = srv.poll(t, len(w), None, want_field=False)
        assert s == F.FEMH_OK
    rep = srv.report()
    assert rep["peak_resident_bytes"] <= 64 << 20
    assert rep["rejected"] == 1 and rep["completed"] == 3
    srv.close()


def test_three_precisions_grouped_match_plain_solves(ctx):
    """Requests of all three precisions resident at once (three iteration
    groups on one stream, members joining and leaving between chunks): each
    field is bit-identical to femh_solve with the same options."""
    reqs = _requests(5, 6, n_hi=16)
    precs = [F.FEMH_FP64, F.FEMH_MIXED_MATRIX, F.FEMH_MIXED] * 2
    srv = F.Server(ctx, max_slots=8, chunk_iters=16)
    tickets = [srv.submit(p, w, precision=pr, rtol=1e-7) for (p, w), pr in zip(reqs, precs)]
    fields = []
    for (p, w), t in zip(reqs, tickets):
        st, H, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert st == F.FEMH_OK, stats
        fields.append((H, stats))
    srv.close()
    for (p, w), pr, (H, stats) in zip(reqs, precs, fields):
        P = F.Problem(ctx, p)
        H1, s1, st1 = P.solve(w, precision=pr, rtol=1e-7, check_every=16)
        assert st1 == F.FEMH_OK
        np.testing.assert_array_equal(H, H1)
        assert [s["iters"] for s in stats] == [s["iters"] for s in s1]
        P.close()


@pytest.mark.parametrize("prec", [F.FEMH_MIXED_MATRIX, F.FEMH_FP64])
def test_batch_rhs_requests_same_alone_in_mix_and_batched(ctx, prec):
    """With batch_rhs, a request's waves are solved in groups of up to four by
    the batched solver: each field is bit-identical alone, in a mix of
    requests that overlap on the device, and to femh_solve_batched_dev on the
    same group of waves; and within 1e-6 of the plain single-RHS solve."""
    import torch
    rng = np.random.default_rng(8)
    reqs = [W.serving_request(rng, n_lo=8, n_hi=16, nrhs_hi=3) for _ in range(5)]
    p6, w6 = W.pec_sphere_batched(n=12, radius=0.3, nrhs=6, seed=12)   # groups of 4 + 2
    reqs.append((p6, w6))
    opts = dict(precision=prec, rtol=1e-7, check_every=16)
    srv = F.Server(ctx, max_slots=8, chunk_iters=16, batch_rhs=True)
    alone = []
    for p, w in reqs[:2]:
        t = srv.submit(p, w, **opts)
        st, H, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert st == F.FEMH_OK, stats
        alone.append(H)
    tickets = [srv.submit(p, w, **opts) for p, w in reqs]
    fields = []
    for (p, w), t in zip(reqs, tickets):
        st, H, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert st == F.FEMH_OK, stats
        fields.append(H)
    assert srv.report()["failed"] == 0
    srv.close()
    for a, H in zip(alone, fields[:2]):
        np.testing.assert_array_equal(a, H)
    for (p, w), H in zip(reqs, fields):
        P = F.Problem(ctx, p)
        if len(w) >= 2:
            for g in range(0, len(w), 4):
                ww = w[g:g + 4]
                out = torch.zeros(P.grid_shape(len(ww)), dtype=torch.complex128, device="cuda")
                s, st = P.solve_dev(ww, out, batched=True, **opts)
                assert st == F.FEMH_OK, s
                np.testing.assert_array_equal(out.cpu().numpy(), H[g:g + 4])
        Hs, s1, st1 = P.solve(w, precision=F.FEMH_FP64, rtol=1e-9)
        assert st1 == F.FEMH_OK
        for r in range(len(w)):
            assert np.linalg.norm(H[r] - Hs[r]) / np.linalg.norm(Hs[r]) <= 1e-6
        P.close()


def test_batch_rhs_cancel_and_admission(ctx):
    """With batch_rhs, a long batched request can be cancelled while the
    others finish; under a small memory budget every batched request is
    still served and the resident bytes (estimates that include the batched
    groups' workspace) never exceed it."""
    big, wbig = W.pec_sphere_batched(n=30, radius=0.8, nrhs=3, seed=9)
    small = [W.serving_request(np.random.default_rng(s), n_lo=8, n_hi=12, nrhs_hi=3) for s in (21, 22, 23)]
    srv = F.Server(ctx, max_slots=4, chunk_iters=16, batch_rhs=True)
    tb = srv.submit(big, wbig, precision=F.FEMH_FP64, rtol=1e-10)
    ts = [srv.submit(p, w, precision=F.FEMH_FP64, rtol=1e-6) for p, w in small]
    assert srv.cancel(tb) == F.FEMH_OK
    st, _, _ = srv.poll(tb, 3, None, want_field=False)
    assert st == F.FEMH_E_CANCELLED
    for (p, w), t in zip(small, ts):
        s, _, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert s == F.FEMH_OK, stats
    srv.close()
    srv = F.Server(ctx, hbm_budget_bytes=96 << 20, max_slots=4, batch_rhs=True)
    ts = [srv.submit(p, w, precision=F.FEMH_FP64, rtol=1e-6) for p, w in small]
    for (p, w), t in zip(small, ts):
        s, _, _ = srv.poll(t, len(w), None, want_field=False)
        assert s == F.FEMH_OK
    rep = srv.report()
    assert rep["peak_resident_bytes"] <= 96 << 20 and rep["completed"] == 3
    srv.close()


# A batched group runs FP64 directions, so FEMH_MIXED with batched waves is the
# complex64-matrix case already listed; it is not repeated.
@pytest.mark.parametrize("prec,batch", [(F.FEMH_FP64, False), (F.FEMH_MIXED_MATRIX, False), (F.FEMH_MIXED, False),
                                        (F.FEMH_FP64, True), (F.FEMH_MIXED_MATRIX, True)])
def test_served_fields_match_the_oracle(ctx, prec, batch):
    """Requests of different sizes served together (they overlap on the
    device) against the CPU oracle: the oracle's scalar assembly, SuperLU
    solution and 1-norm condition estimate, the solve tolerance chosen as
    0.1 * target / kappa so that the forward error is certified below the
    target (1e-9 FP64, 1e-6 mixed).  Each field must match the oracle's at
    every active node to the target and be exactly zero at the nodes of PEC
    elements only."""
    from oracle import fem, solve

    target = 1e-9 if prec == F.FEMH_FP64 else 1e-6
    reqs = _requests(31, 4, n_hi=12)
    refs = []
    for p, w in reqs:
        A = fem.assemble(p)
        X = solve.sparse_solve(A, fem.rhs(p, w))
        kappa = solve.condest(A)
        refs.append((fem.scatter_to_grid(p, X), min(1e-7, 0.1 * target / kappa), fem.Mesh(p).node_active))
    srv = F.Server(ctx, max_slots=8, chunk_iters=16, batch_rhs=batch)
    tickets = [srv.submit(p, w, precision=prec, rtol=rtol) for (p, w), (_, rtol, _) in zip(reqs, refs)]
    for (p, w), t, (Ho, rtol, active) in zip(reqs, tickets, refs):
        st, H, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert st == F.FEMH_OK, stats
        for r in range(len(w)):
            err = np.linalg.norm(H[r] - Ho[r]) / np.linalg.norm(Ho[r])
            assert err <= target, (prec, batch, r, err, rtol, stats[r])
            assert stats[r]["rel_residual"] <= rtol
        assert np.all(H[:, ~active] == 0)
    rep = srv.report()
    assert rep["failed"] == 0 and rep["completed"] == len(reqs)
    srv.close()


def test_many_batched_requests_at_once_match_batched_solves(ctx):
    """Twenty-four requests with batched waves submitted together, so that
    set-up (assembly, graph capture) of some overlaps the iterations of
    others: every request succeeds, and each group of up to four waves is
    bit-identical to femh_solve_batched_dev on the same waves."""
    import torch
    rng = np.random.default_rng(17)
    reqs = [W.serving_request(rng, n_lo=8, n_hi=16, nrhs_hi=9) for _ in range(24)]
    opts = dict(precision=F.FEMH_FP64, rtol=1e-6, check_every=16)
    srv = F.Server(ctx, max_slots=16, chunk_iters=16, batch_rhs=True)
    tickets = [srv.submit(p, w, **opts) for p, w in reqs]
    fields = []
    for (p, w), t in zip(reqs, tickets):
        st, H, stats = srv.poll(t, len(w), _shape(p, len(w)))
        assert st == F.FEMH_OK, stats
        fields.append(H)
    rep = srv.report()
    assert rep["completed"] == len(reqs) and rep["failed"] == 0
    srv.close()
    for (p, w), H in zip(reqs, fields):
        P = F.Problem(ctx, p)
        for g in range(0, len(w), 4):
            ww = w[g:g + 4]
            out = torch.zeros(P.grid_shape(len(ww)), dtype=torch.complex128, device="cuda")
            # a request of two or more waves runs every group (a last group
            # of one included) through the batched solver
            s, st = P.solve_dev(ww, out, batched=len(w) >= 2, **opts)
            assert st == F.FEMH_OK, s
            np.testing.assert_array_equal(out.cpu().numpy(), H[g:g + 4])
        P.close()
