"""Request server (continuous batching) against plain searches, through the C ABI."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1703_05581_amd import ffa, synth

    assert torch.cuda.is_available()
    return torch, ffa, synth


def _footprint(plan, host: bool) -> int:
    up = lambda v: -(-v // 256) * 256  # noqa: E731
    series = plan.N * (1 if plan.dtype == "u8" else 4)
    return (up(series) if host else 0) + up(plan.ws_bytes) + 2 * up(plan.n_trials * 4)


def _reference(torch, plan, x):
    xt = torch.from_numpy(x).cuda()
    s, w = plan.search(xt)
    torch.cuda.synchronize()
    return s.cpu().numpy(), w.cpu().numpy()


def test_server_matches_search(env):
    """A mix of uint8 / float32, host / device inputs and plans: every
    periodogram equals the plain search's, bit for bit."""
    torch, ffa, synth = env
    plans = [ffa.Plan(60000, 1e-3, 0.2, 0.9, 200, W10, "u8"),
             ffa.Plan(90000, 1e-3, 0.3, 1.5, 256, None, "f32"),
             ffa.Plan(1 << 18, 1e-3, 0.256, 2.048, 256, W10, "u8")]
    srv = ffa.Server(4 << 30, 4)
    jobs = []
    for i in range(12):
        p = plans[i % 3]
        x = synth.random_series(900 + i, p.N, p.dtype)
        arg = torch.from_numpy(x).cuda() if i % 4 == 3 else x
        jobs.append((srv.submit(p, arg), p, x, arg))
    for t, p, x, _ in jobs:
        print("ticket", t, flush=True)
        s, w, lat = srv.wait(t)
        s0, w0 = _reference(torch, p, x)
        assert np.array_equal(s, s0) and np.array_equal(w, w0), t
        assert 0 < lat < 60
    srv.close()


def test_server_admission_timeout_and_errors(env):
    """A pool that fits one request admits the next only after the first is
    collected; polling a queued request times out; bad tickets and oversize
    requests are refused."""
    torch, ffa, synth = env
    p = ffa.Plan(100000, 1e-3, 0.2, 1.0, 200, W10, "u8")
    fp = _footprint(p, host=True)
    srv = ffa.Server(fp + 4096, 2)
    xs = [synth.random_series(40 + i, p.N, "u8") for i in range(3)]
    tickets = [srv.submit(p, x) for x in xs]
    with pytest.raises(ffa.FFAError) as e:
        srv.wait(tickets[2], timeout_s=0)  # cannot run before ticket 1 is collected
    assert e.value.status == ffa.FFA_ERR_TIMEOUT
    for t, x in zip(tickets, xs):
        s, w, _ = srv.wait(t)
        s0, w0 = _reference(torch, p, x)
        assert np.array_equal(s, s0) and np.array_equal(w, w0)
    lib = ffa.lib()
    assert lib.ffa_server_wait(srv._h, tickets[0], 0, None, None, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_wait(srv._h, 12345, 0, None, None, None) == ffa.FFA_ERR_INVALID
    big = ffa.Plan(1 << 20, 1e-3, 0.256, 2.048, 256, W10, "u8")
    with pytest.raises(ffa.FFAError) as e:
        srv.submit(big, synth.random_series(1, 1 << 20, "u8"))
    assert e.value.status == ffa.FFA_ERR_UNSUPPORTED
    srv.close()


def test_server_concurrent_clients(env):
    """Four client threads submit and collect at once."""
    torch, ffa, synth = env
    p = ffa.Plan(50000, 1e-3, 0.2, 0.8, 128, W10, "f32")
    srv = ffa.Server(1 << 30, 3)
    xs = [synth.random_series(70 + i, p.N, "f32") for i in range(12)]
    refs = [_reference(torch, p, x) for x in xs]
    errors = []

    def client(k):
        try:
            mine = [(srv.submit(p, xs[i]), i) for i in range(k, 12, 4)]
            for t, i in mine:
                s, w, _ = srv.wait(t)
                if not (np.array_equal(s, refs[i][0]) and np.array_equal(w, refs[i][1])):
                    errors.append(i)
        except Exception as exc:  # noqa: BLE001
            errors.append(repr(exc))

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors
    srv.close()


def test_server_failure_isolation(env):
    """A request whose launch fails (forced on the host by the test hook,
    before anything of it is enqueued) reports FFA_ERR_DEVICE; every other
    request, before and after it, is served bit for bit, and the server keeps
    admitting afterwards."""
    torch, ffa, synth = env
    plans = [ffa.Plan(60000, 1e-3, 0.2, 0.9, 200, W10, "u8"),
             ffa.Plan(80000, 1e-3, 0.3, 1.5, 256, None, "f32")]
    srv = ffa.Server(2 << 30, 3)
    srv.fail_ticket(4)  # tickets are issued from 1 in submission order
    jobs = []
    for i in range(8):
        p = plans[i % 2]
        x = synth.random_series(1200 + i, p.N, p.dtype)
        jobs.append((srv.submit(p, x), p, x))
    assert [t for t, _, _ in jobs] == list(range(1, 9))
    for t, p, x in jobs:
        print("ticket", t, flush=True)
        if t == 4:
            with pytest.raises(ffa.FFAError) as e:
                srv.wait(t)
            assert e.value.status == ffa.FFA_ERR_DEVICE
            continue
        s, w, _ = srv.wait(t)
        s0, w0 = _reference(torch, p, x)
        assert np.array_equal(s, s0) and np.array_equal(w, w0), t
    x = synth.random_series(1300, plans[0].N, "u8")
    s, w, _ = srv.wait(srv.submit(plans[0], x))
    s0, w0 = _reference(torch, plans[0], x)
    assert np.array_equal(s, s0) and np.array_equal(w, w0)
    srv.close()


def _backfill_setup(ffa):
    big = ffa.Plan(200000, 1e-3, 0.2, 1.0, 200, W10, "u8")
    small = ffa.Plan(30000, 1e-3, 0.2, 0.6, 200, W10, "u8")
    fb, fs = _footprint(big, True), _footprint(small, True)
    assert fb > fs + 8192 and fs > 8192
    return big, small, fb + fs + 4096  # one big and one small fit, no more


def test_server_strict_order(env):
    """max_bypass 0: a small request behind a big one that does not fit
    waits, though it would fit."""
    torch, ffa, synth = env
    big, small, budget = _backfill_setup(ffa)
    srv = ffa.Server(budget, 2, max_bypass=0)
    xb = [synth.random_series(60 + i, big.N, "u8") for i in range(2)]
    xs = synth.random_series(70, small.N, "u8")
    tb = [srv.submit(big, x) for x in xb]
    ts = srv.submit(small, xs)
    with pytest.raises(ffa.FFAError) as e:
        srv.wait(ts, timeout_s=0.3)
    assert e.value.status == ffa.FFA_ERR_TIMEOUT
    for t, p, x in [(tb[0], big, xb[0]), (tb[1], big, xb[1]), (ts, small, xs)]:
        s, w, _ = srv.wait(t)
        s0, w0 = _reference(torch, p, x)
        assert np.array_equal(s, s0) and np.array_equal(w, w0), t
    srv.close()


def test_server_backfill_and_aging_bound(env):
    """max_bypass 1: the first small request passes the blocked big one; once
    it has, the second small waits for the big one although it would fit."""
    torch, ffa, synth = env
    big, small, budget = _backfill_setup(ffa)
    srv = ffa.Server(budget, 2, max_bypass=1)
    xb = [synth.random_series(80 + i, big.N, "u8") for i in range(2)]
    xs = [synth.random_series(90 + i, small.N, "u8") for i in range(2)]
    tb = [srv.submit(big, x) for x in xb]
    ts = [srv.submit(small, x) for x in xs]
    s, w, _ = srv.wait(ts[0], timeout_s=60)  # admitted past the blocked head
    s0, w0 = _reference(torch, small, xs[0])
    assert np.array_equal(s, s0) and np.array_equal(w, w0)
    with pytest.raises(ffa.FFAError) as e:  # fits now, but the head was passed once
        srv.wait(ts[1], timeout_s=0.3)
    assert e.value.status == ffa.FFA_ERR_TIMEOUT
    for t, p, x in [(tb[0], big, xb[0]), (tb[1], big, xb[1]), (ts[1], small, xs[1])]:
        s, w, _ = srv.wait(t)
        s0, w0 = _reference(torch, p, x)
        assert np.array_equal(s, s0) and np.array_equal(w, w0), t
    srv.close()


def test_server_device_input_after_producer_stream(env):
    """A device series written by work still queued on the caller's stream
    at submission is read only after that work: the request's stream waits
    on an event recorded on the producer stream."""
    torch, ffa, synth = env
    p = ffa.Plan(1 << 18, 1e-3, 0.256, 2.048, 256, W10, "u8")
    x_np = synth.random_series(1400, p.N, "u8")
    src = torch.from_numpy(x_np).cuda()
    dst = torch.zeros_like(src)
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    srv = ffa.Server(2 << 30, 2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for _ in range(20):  # keep the producer stream busy ahead of the copy
            a = torch.mm(a, a).clamp_(-1.0, 1.0)
        dst.copy_(src)
        t = srv.submit(p, dst)
    s, w, _ = srv.wait(t)
    torch.cuda.synchronize()
    s0, w0 = _reference(torch, p, x_np)
    assert np.array_equal(s, s0) and np.array_equal(w, w0)
    srv.close()
