"""GPU tests of graph lists and of the continuous-batching server: every
request's labels equal the CPU oracle's and the same request solved alone,
whatever it was batched with; admission by device footprint queues work
instead of failing; errors stay with the request that caused them."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

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
        tickets = [srv.submit(u, v, n) for u, v, n in reqs]
        results = [srv.wait(t) for t in tickets]
        assert srv.stats()["arena_used"] == 0
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
