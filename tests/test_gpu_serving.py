"""GPU tests of graph lists and of the continuous-batching server: every
request's labels equal the CPU oracle's and the same request solved alone,
whatever it was batched with; admission by device footprint queues work
instead of failing; errors stay with the request that caused them."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests.golden import cases

torch = pytest.importorskip("torch")
import paper_1612_01178_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cc.load()
    return torch.device("cuda:0")


def _requests(count, seed, scale_hi=17):
    sc, ef = graphgen.serving_request_shapes(count, seed=seed, scale_lo=6, scale_hi=scale_hi,
                                             ef_lo=1, ef_hi=20)
    out = []
    for i in range(count):
        u, v, n = graphgen.serving_request(i, int(sc[i]), int(ef[i]), seed=seed)
        out.append((u, v, n))
    return out


def test_graph_list_matches_oracle_and_solo(dev):
    reqs = _requests(40, seed=77, scale_hi=18)
    reqs.append((np.zeros(0, np.int32), np.zeros(0, np.int32), 5))  # no edges
    reqs.append((np.zeros(0, np.int32), np.zeros(0, np.int32), 0))  # empty graph
    tens = [(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev), n) for u, v, n in reqs]
    say("graph list of", len(tens))
    outs, st = cc.labels_list(tens, return_stats=True)
    assert st["host_syncs"] == 1
    for (u, v, n), (du, dv, _), got in zip(reqs, tens, outs):
        want = oracle.labels(u, v, n)
        assert np.array_equal(got.cpu().numpy(), want)
        solo = cc.labels(du, dv, n).cpu().numpy()
        assert np.array_equal(solo, want)


def test_server_mix_equals_alone_device_requests(dev):
    reqs = _requests(48, seed=91, scale_hi=18)
    tens = [(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev), n) for u, v, n in reqs]
    with cc.Server(workers=3, max_batch=16) as srv:
        say("server: submitting", len(tens), "device requests at once")
        tickets = [srv.submit(du, dv, n) for du, dv, n in tens]
        results = [srv.wait(t) for t in tickets]
        assert srv.stats()["pending"] == 0
    batched = 0
    for (u, v, n), (du, dv, _), (lab, info) in zip(reqs, tens, results):
        assert info["status"] == 0
        assert info["t_submit"] <= info["t_admit"] <= info["t_launch"] <= info["t_device_done"]
        batched += info["batch_size"] > 1
        want = oracle.labels(u, v, n)
        assert np.array_equal(lab.cpu().numpy(), want)
        assert np.array_equal(cc.labels(du, dv, n).cpu().numpy(), want)
    assert batched > 0, "no request shared a wave"


def test_server_host_requests_queue_on_small_arena(dev):
    reqs = _requests(24, seed=5, scale_hi=16)
    biggest = max(2 * len(u) * 4 + 4 * n for u, v, n in reqs)
    arena = biggest * 2 + 4096
    with cc.Server(device_bytes=arena, workers=2) as srv:
        say("server: host requests, arena", arena)
        fixed = srv.stats()["arena_used"]  # the workers' own workspace blocks
        assert 0 < fixed < 1 << 20
        tickets = [srv.submit(u, v, n) for u, v, n in reqs]
        results = [srv.wait(t) for t in tickets]
        assert srv.stats()["arena_used"] == fixed
    for (u, v, n), (lab, info) in zip(reqs, results):
        assert info["status"] == 0 and info["t_host_done"] >= info["t_device_done"]
        assert np.array_equal(lab, oracle.labels(u, v, n))


def test_server_errors_stay_with_their_request(dev):
    good = _requests(6, seed=13, scale_hi=12)
    with cc.Server(device_bytes=1 << 20, workers=1, max_batch=64) as srv:
        bad_u = np.array([0, 1, 9], np.int32)
        bad_v = np.array([1, 2, 3], np.int32)
        tb = srv.submit(bad_u, bad_v, 5)  # endpoint 9 outside [0, 5)
        big = srv.submit(np.zeros(1 << 18, np.int32), np.zeros(1 << 18, np.int32), 4)
        tg = [srv.submit(u, v, n) for u, v, n in good]
        with pytest.raises(cc.CCError) as ei:
            srv.wait(tb)
        assert ei.value.code == cc.CC_ERR_RANGE
        with pytest.raises(cc.CCError) as ei:
            srv.wait(big)  # 2 MiB of edges never fits the 1 MiB arena
        assert ei.value.code == cc.CC_ERR_NOMEM
        for (u, v, n), t in zip(good, tg):
            lab, info = srv.wait(t)
            assert np.array_equal(lab, oracle.labels(u, v, n))


def test_concurrent_calls_from_host_threads(dev):
    """Calls from several host threads on their own streams at once (the
    workspace cache is per stream) give the same labels as alone."""
    import threading
    reqs = _requests(12, seed=31, scale_hi=17)
    want = [oracle.labels(u, v, n) for u, v, n in reqs]
    tens = [(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev), n) for u, v, n in reqs]
    torch.cuda.synchronize()
    results = [None] * len(reqs)
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(3):
                    for i in range(k, len(tens), 4):
                        du, dv, n = tens[i]
                        lab = cc.labels(du, dv, n, stream=s,
                                        options=cc.Options(hook=("atomic", "plain", "auto")[rep]))
                        s.synchronize()
                        results[i] = lab.cpu().numpy()
                        assert np.array_equal(results[i], want[i]), (i, rep)
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i in range(len(reqs)):
        assert np.array_equal(results[i], want[i])


SERVING_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                              "serving_digests.json")


def _digest(lab):
    return hashlib.sha256(np.ascontiguousarray(lab, dtype="<i4").tobytes()).hexdigest()


def _mix_requests():
    gold = json.load(open(SERVING_GOLDEN))["mix"]
    spec = cases.serving_mix()
    assert [(r["index"], r["scale"], r["edge_factor"]) for r in gold["requests"]] == spec
    reqs = []
    for (i, sc, ef), rec in zip(spec, gold["requests"]):
        u, v, n = graphgen.serving_request(i, sc, ef, seed=cases.SERVING_MIX_SEED)
        assert (n, len(u)) == (rec["n"], rec["m"])
        reqs.append((u, v, n, rec["sha256"]))
    return reqs


def test_server_at_serving_sizes_matches_oracle_and_solo(dev):
    """The serving workload's sizes: requests at R-MAT scale 19-22 with edge
    factor 21-32 (up to 2^27 entries: the large-request path, several at once
    on 3 worker streams) mixed with small ones, half with device-resident
    arrays and half with host arrays; every result equals the oracle's
    (digest) and the same request solved alone."""
    say("serving mix: generating")
    reqs = _mix_requests()
    say("serving mix:", len(reqs), "requests,", sum(len(r[0]) for r in reqs), "entries")
    dreqs = {}
    for k, (u, v, n, _) in enumerate(reqs):
        if k % 2 == 0:
            dreqs[k] = (torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev))
    with cc.Server(workers=3, max_batch=64) as srv:
        tickets = []
        for k, (u, v, n, _) in enumerate(reqs):
            tickets.append(srv.submit(*dreqs[k], n) if k in dreqs else srv.submit(u, v, n))
        results = [srv.wait(t) for t in tickets]
    spans = []
    for k, ((u, v, n, sha), (lab, info)) in enumerate(zip(reqs, results)):
        assert info["status"] == 0
        got = lab.cpu().numpy() if k in dreqs else lab
        assert _digest(got) == sha, ("request", k, n, len(u))
        du, dv = dreqs[k] if k in dreqs else (torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev))
        assert np.array_equal(cc.labels(du, dv, n).cpu().numpy(), got), ("solo", k)
        if n > cc.CC_BATCH_LDS_MAX_N:
            spans.append((info["t_launch"], info["t_device_done"]))
    overlaps = sum(1 for i, a in enumerate(spans) for b in spans[i + 1:]
                   if a[0] < b[1] and b[0] < a[1])
    say("serving mix: large requests whose solves overlapped in time (pairs):", overlaps)


def test_server_budget_queues_large_requests(dev):
    """A 1 GiB footprint budget: four large requests (8m + 4n + workspace of
    150-500 MB each, 1.24 GB together) cannot all be admitted at once, so
    the later ones wait for earlier ones to finish instead of failing; a
    request whose footprint exceeds the budget fails with CC_ERR_NOMEM."""
    reqs = _mix_requests()
    pick = [1, 5, 2, 3]  # scale/ef (21, 28), (21, 22), (20, 21), (19, 30)
    tens = {k: (torch.from_numpy(reqs[k][0]).to(dev), torch.from_numpy(reqs[k][1]).to(dev))
            for k in pick + [0]}
    with cc.Server(device_bytes=1 << 30, workers=3) as srv:
        say("budget test: submitting", pick)
        tickets = [srv.submit(*tens[k], reqs[k][2]) for k in pick]
        too_big = srv.submit(*tens[0], reqs[0][2])  # (22, 32): 8m alone is 1.07 GB
        results = [srv.wait(t) for t in tickets]
        with pytest.raises(cc.CCError) as ei:
            srv.wait(too_big)
        assert ei.value.code == cc.CC_ERR_NOMEM
    infos = [info for _, info in results]
    for k, (lab, info) in zip(pick, results):
        assert info["status"] == 0
        assert _digest(lab.cpu().numpy()) == reqs[k][3]
    # some request was admitted only after another one had finished
    first_done = min(i["t_device_done"] for i in infos)
    assert max(i["t_admit"] for i in infos) >= first_done


def test_server_waits_for_the_producer_stream(dev):
    """Edges written by work still queued on a side stream when the request
    is submitted: the worker's stream waits for that point of the side
    stream before reading them."""
    u, v, n = graphgen.rmat(16, 8, seed=4141)
    want = oracle.labels(u, v, n)
    src_u = torch.from_numpy(u).to(dev)
    src_v = torch.from_numpy(v).to(dev)
    du = torch.zeros_like(src_u)  # all-(0, 0) edges until the copies land
    dv = torch.zeros_like(src_v)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with cc.Server(workers=2) as srv:
        with torch.cuda.stream(side):
            a = torch.randn(4096, 4096, device=dev)
            for _ in range(30):  # tens of ms of queued work ahead of the copies
                a = a @ a
                a = a / a.norm()
            du.copy_(src_u)
            dv.copy_(src_v)
            t = srv.submit(du, dv, n, stream=side)
        lab, info = srv.wait(t)
        side.synchronize()
    assert info["status"] == 0
    assert np.array_equal(lab.cpu().numpy(), want)
