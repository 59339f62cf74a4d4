"""Serving engine: memory admission, overlap, and results identical alone and in the mix."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

MARGIN = 260   # output margin at R0 = 1e6 (rotation + RV + 6 sigma IP reach < 200 points)


@pytest.fixture(scope="module")
def setup():
    from paper_2105_14782_amd import api
    lists, nu = synth.serving_pool(n_lists=6, min_lines=300, max_lines=6000)
    ctx = api.Context(0)
    for s, ll in enumerate(lists):
        ctx.set_lines(s, ll)
    ctx.set_grid(nu)
    reqs = synth.serving_requests(24, rate_hz=0.0, n_lists=6, nu_master=nu, min_grid=2000,
                                  max_grid=8000, min_layers=20, max_layers=60)
    return api, ctx, lists, nu, reqs


def _req_args(api, nu, lists, q):
    P, T0, al, logx, rv, vs = synth.serving_atmosphere(q)
    u1, u2 = 0.5366563145999494, 0.35777087639996635
    atm = api.Atmos(P, T0, al, list(q.species), list(logx), cia_alpha0=5e-46, cia_Tpow=1.0,
                    cia_slope=0.1, cia_nu_c=4500.0, vmr_h2=0.75 * 2.33 / 2.016,
                    grid_begin=q.grid_begin, grid_len=q.grid_len)
    resp = api.Response(rv, vs, u1, u2, 1e5, MARGIN, q.grid_len - 2 * MARGIN)
    return atm, resp


def test_results_identical_alone_and_in_mix(setup):
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    args = [_req_args(api, nu, lists, q) for q in reqs]
    # alone: one slot, each request waited for before the next is submitted
    alone = serve.Server(ctx, n_streams=1, mem_budget_bytes=4 << 30)
    ref = []
    for a, r in args:
        t = alone.submit(a, r)
        ref.append(alone.wait(t).flux.cpu())
    alone.close()
    # mix: four slots, everything submitted at once
    mix = serve.Server(ctx, n_streams=4, mem_budget_bytes=4 << 30)
    out = serve.run_stream(mix, args)
    st = mix.stats()
    mix.close()
    assert st["completed"] == len(args) and st["failed"] == 0
    assert st["mem_peak_bytes"] <= st["mem_budget_bytes"]
    for k, (res, r0) in enumerate(zip(out["results"], ref)):
        assert torch.equal(res.flux.cpu(), r0), k
    # and the synchronous API gives the same spectrum
    a, r = args[3]
    assert torch.equal(ctx.emission_flux(a, r).cpu(), ref[3])


def test_hundred_requests_identical_alone_and_in_mix(setup):
    """100 requests with the serving workload's layer counts (50-200) and
    windows of 2,000-20,000 points: each result is bitwise the one it gives
    alone, with eight slots and every request submitted at once."""
    api, ctx, lists, nu, _ = setup
    from paper_2105_14782_amd import serve
    reqs = synth.serving_requests(100, rate_hz=0.0, seed=2024, n_lists=6, nu_master=nu,
                                  min_grid=2000, max_grid=20000, min_layers=50, max_layers=200)
    args = [_req_args(api, nu, lists, q) for q in reqs]
    ref = [ctx.emission_flux(a, r).cpu() for a, r in args]
    mix = serve.Server(ctx, n_streams=8, mem_budget_bytes=8 << 30)
    out = serve.run_stream(mix, args)
    st = mix.stats()
    mix.close()
    print(f"  100 requests: peak in flight {st['peak_in_flight']}, "
          f"{out['spectra_per_s']:.1f} spectra/s", flush=True)
    assert st["completed"] == len(args) and st["failed"] == 0
    assert st["peak_in_flight"] >= 2
    same = [torch.equal(res.flux.cpu(), r0) for res, r0 in zip(out["results"], ref)]
    assert all(same), [k for k, s in enumerate(same) if not s]


def test_fp64_requests_identical_to_the_synchronous_api(setup):
    """FP64 requests in the serving engine give the synchronous FP64 spectrum bitwise."""
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    args = [_req_args(api, nu, lists, q) for q in reqs[:6]]
    ref = [ctx.emission_flux(a, r, "fp64").cpu() for a, r in args]
    srv = serve.Server(ctx, n_streams=3, mem_budget_bytes=4 << 30)
    out = serve.run_stream(srv, args, precision="fp64")
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(args) and st["failed"] == 0
    for k, (res, r0) in enumerate(zip(out["results"], ref)):
        assert res.flux.dtype == torch.float64
        assert torch.equal(res.flux.cpu(), r0), k


def test_serving_result_matches_oracle(setup):
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    q = min(reqs, key=lambda x: x.grid_len * x.n_layers)
    a, r = _req_args(api, nu, lists, q)
    srv = serve.Server(ctx, n_streams=2, mem_budget_bytes=2 << 30)
    F = srv.wait(srv.submit(a, r)).flux.cpu().double().numpy()
    srv.close()
    # oracle on the same window and atmosphere
    wl = synth.Workload("serve", [lists[q.species[0]], lists[q.species[1]]],
                        nu[q.grid_begin:q.grid_begin + q.grid_len],
                        synth.Atmosphere(a.P_bar, a.T0, a.alpha, np.asarray(a.log10_mmr), cia_nu_c=4500.0),
                        synth.Response(r.rv_kms, r.vsini_kms, r.u1, r.u2, r.R_inst, r.out_begin, r.out_len))
    th = np.array([a.T0, a.alpha, *a.log10_mmr, r.rv_kms, r.vsini_kms])
    ref = O.emission_flux(wl, th)
    assert np.max(np.abs(F - ref) / np.abs(ref)) < 1e-4


def test_memory_admission_bounds_and_rejects(setup):
    api, ctx, lists, nu, reqs = setup
    import paper_2105_14782_amd as pkg
    from paper_2105_14782_amd import serve
    args = [_req_args(api, nu, lists, q) for q in reqs[:12]]
    srv = serve.Server(ctx, n_streams=4, mem_budget_bytes=64 << 20)
    need = [srv.workspace_bytes(a, r) for a, r in args]
    fits = [i for i, b in enumerate(need) if b <= (64 << 20)]
    too_big = [i for i, b in enumerate(need) if b > (64 << 20)]
    for i in too_big:
        with pytest.raises(pkg.ExoError) as e:
            srv.submit(*args[i])
        assert e.value.code == pkg.EXO_ENOMEM
    out = serve.run_stream(srv, [args[i] for i in fits])
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(fits)
    assert st["rejected"] == len(too_big)
    assert st["mem_peak_bytes"] <= 64 << 20


def _warm(api, ctx, nu, lists, reqs):
    from paper_2105_14782_amd import serve
    srv = serve.Server(ctx, n_streams=4, mem_budget_bytes=4 << 30)
    serve.run_stream(srv, [_req_args(api, nu, lists, q) for q in reqs])
    srv.close()


def test_requests_overlap_on_the_device(setup):
    """A fixed set of 12 requests: served four at a time they are on the
    device together (peak in-flight >= 2) and finish in less wall time than
    the sum of their times served one at a time."""
    import time
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    _warm(api, ctx, nu, lists, reqs[:12])
    args = [_req_args(api, nu, lists, q) for q in reqs[:12]]
    alone = serve.Server(ctx, n_streams=1, mem_budget_bytes=4 << 30)
    solo = []
    for a, r in args:
        t = time.monotonic()
        alone.wait(alone.submit(a, r))
        solo.append(time.monotonic() - t)
    alone.close()
    mix = serve.Server(ctx, n_streams=4, mem_budget_bytes=4 << 30)
    out = serve.run_stream(mix, args)
    st = mix.stats()
    mix.close()
    print(f"  sum of solo times {1e3 * sum(solo):.1f} ms, mixed wall {1e3 * out['wall_s']:.1f} ms, "
          f"peak in flight {st['peak_in_flight']}", flush=True)
    assert st["peak_in_flight"] >= 2
    assert out["wall_s"] < sum(solo)


def test_small_requests_bypass_a_head_waiting_for_memory(setup):
    """While a large request waits for memory at the head of the queue,
    smaller requests that fit are admitted ahead of it, at most 8 of them; the
    rest wait for it.  Every result is still the one the request gives alone."""
    import time
    from dataclasses import replace
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    big = replace(reqs[0], grid_begin=2000, grid_len=150000, n_layers=200)
    A = _req_args(api, nu, lists, big)
    H = _req_args(api, nu, lists, replace(big, theta=reqs[1].theta))
    small = [_req_args(api, nu, lists, replace(q, grid_len=2000, n_layers=20)) for q in reqs[2:14]]
    probe = serve.Server(ctx, n_streams=1, mem_budget_bytes=1 << 20)
    wa = max(probe.workspace_bytes(*A), probe.workspace_bytes(*H))
    ws = max(probe.workspace_bytes(*s) for s in small)
    probe.close()
    budget = wa + wa // 2
    assert 3 * ws < wa // 2, (ws, wa)   # three small requests fit beside the first large one
    ref = [ctx.emission_flux(*x).cpu() for x in [A, H] + small]
    srv = serve.Server(ctx, n_streams=4, mem_budget_bytes=budget)
    t0 = time.monotonic()    # one arrival instant for all: queue times order the admissions
    tickets = [srv.submit(a, r, arrival_s=t0) for a, r in [A, H] + small]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    ahead = sum(r.queue_s < res[1].queue_s for r in res[2:])
    print(f"  bypasses {st['bypasses']}, small requests admitted before the waiting head {ahead}",
          flush=True)
    assert 1 <= st["bypasses"] <= 8
    assert ahead == st["bypasses"]
    for k, (r, f) in enumerate(zip(res, ref)):
        assert torch.equal(r.flux.cpu(), f), k


def test_full_scale_serving_requests_against_oracle():
    """The serving workload at its full scale: the resident pool of 16 lists
    (1e3-1e6 lines over 3900-5100 cm^-1) on the R0 = 1e6 master grid, and the
    three largest of 40 requests drawn from its arrival process (by line x
    point x layer count), served together without the response.  Each F0 at
    64 sampled points (both window ends and 62 random ones) against the
    oracle over all lines and layers."""
    import time
    from paper_2105_14782_amd import api, serve
    lists, nu = synth.serving_pool()
    ctx = api.Context(0)
    for s, ll in enumerate(lists):
        ctx.set_lines(s, ll)
    ctx.set_grid(nu)
    pool = synth.serving_requests(40, rate_hz=0.0, seed=4242, nu_master=nu)
    work = [(lists[q.species[0]].n + lists[q.species[1]].n) * q.grid_len * q.n_layers for q in pool]
    reqs = [pool[k] for k in np.argsort(work)[-3:]]
    args = []
    for q in reqs:
        P, T0, al, logx, rv, vs = synth.serving_atmosphere(q)
        args.append(api.Atmos(P, T0, al, list(q.species), list(logx), cia_alpha0=5e-46, cia_Tpow=1.0,
                              cia_slope=0.1, cia_nu_c=4500.0, vmr_h2=0.75 * 2.33 / 2.016,
                              grid_begin=q.grid_begin, grid_len=q.grid_len))
    srv = serve.Server(ctx, n_streams=3, mem_budget_bytes=48 << 30)
    tickets = [srv.submit(a, None) for a in args]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 3 and st["failed"] == 0
    rng = np.random.default_rng(4243)
    for q, a, r in zip(reqs, args, res):
        F = r.flux.cpu().double().numpy()
        idx = np.concatenate([[0], np.sort(rng.choice(np.arange(1, q.grid_len - 1), 62, replace=False)),
                              [q.grid_len - 1]])
        wl = synth.Workload("serve-full", [lists[q.species[0]], lists[q.species[1]]],
                            nu[q.grid_begin:q.grid_begin + q.grid_len],
                            synth.Atmosphere(a.P_bar, a.T0, a.alpha, np.asarray(a.log10_mmr), cia_nu_c=4500.0),
                            None)
        t = time.monotonic()
        ref = O.emission_F0(wl, np.array([a.T0, a.alpha, *a.log10_mmr]), nu_idx=idx)
        err = float(np.max(np.abs(F[idx] - ref) / np.abs(ref)))
        print(f"  {lists[q.species[0]].n + lists[q.species[1]].n} lines x {q.grid_len} points x "
              f"{q.n_layers} layers: max rel err {err:.2e} (oracle {time.monotonic() - t:.1f} s)", flush=True)
        assert err < 1e-4
    ctx.close()


def test_shortest_first_policy_order_and_pass_bound(setup):
    """With the shortest-first policy and max_passes = 1 on one slot: while a
    large request runs, a second large one and three small ones queue.  The
    admissions follow the rule (the fewest evaluations first, but a request
    passed over once is preferred next), which puts the large one second,
    not last; results are bitwise those of the synchronous API."""
    import time
    from dataclasses import replace
    api, ctx, lists, nu, reqs = setup
    from paper_2105_14782_amd import serve
    big = replace(reqs[0], grid_begin=2000, grid_len=150000, n_layers=200)
    qs = [replace(big, theta=reqs[1].theta)] + [replace(q, grid_len=n, n_layers=20)
                                                for q, n in zip(reqs[2:5], (3000, 2000, 4000))]
    args = [_req_args(api, nu, lists, q) for q in [big] + qs]
    work = [(lists[q.species[0]].n + lists[q.species[1]].n) * q.grid_len * q.n_layers for q in qs]
    # the rule, applied to the four queued requests (arrival order = list order)
    queue, passed, expect = list(range(4)), [0] * 4, []
    while queue:
        forced = [k for k in queue if passed[k] >= 1]
        pick = forced[0] if forced else min(queue, key=lambda k: (work[k], k))
        for k in queue[:queue.index(pick)]:
            passed[k] += 1
        queue.remove(pick)
        expect.append(pick + 1)
    srv = serve.Server(ctx, n_streams=1, mem_budget_bytes=8 << 30)
    srv.set_policy("shortest", max_passes=1)
    t0 = time.monotonic()
    tickets = [srv.submit(*args[0], arrival_s=t0)]
    for _ in range(2000):            # the first request holds the slot before the others queue
        if srv.stats()["admitted"] >= 1:
            break
        time.sleep(0.001)
    tickets += [srv.submit(a, r, arrival_s=t0) for a, r in args[1:]]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    order = [int(k) for k in np.argsort([r.queue_s for r in res], kind="stable")]
    print(f"  work {work}; admission order {order}, expected {[0] + expect}", flush=True)
    assert st["completed"] == 5 and st["failed"] == 0
    assert order == [0] + expect
    assert expect.index(1) < 3          # the large request was not left to the end
    for k, ((a, r), x) in enumerate(zip(args, res)):
        assert torch.equal(x.flux.cpu(), ctx.emission_flux(a, r).cpu()), k
    import paper_2105_14782_amd as pkg
    bad = serve.Server(ctx, n_streams=1, mem_budget_bytes=1 << 20)
    with pytest.raises(pkg.ExoError):
        bad.set_policy("shortest", max_passes=0)
    bad.close()
