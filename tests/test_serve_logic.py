"""Scheduling logic of the solve server on the CPU, with a stand-in backend
that follows the same leg-dim schedule as HOTRG and completes steps after a
fixed number of polls (no GPU, no kernels)."""
import pytest

from paper_1911_12954_amd.serve import Server
from trg_inputs import serving_requests


class FakeHandle:
    def __init__(self, req):
        self.req = req
        self.dims = [2, 2, 2, 2]
        self.steps = 0


class FakeBackend:
    """Resident bytes grow like D^8, a lane's workspace like D^9; a lane's
    step completes after `lag` polls."""

    def __init__(self, lag=2):
        self.lag = lag
        self.live = 0
        self.max_live = 0
        self.calls = []
        self.workspaces = {}     # id of the first run of a lane's workspace -> users
        self.max_workspaces = 0

    def resident(self, req):
        return 10 * req["dcut"] ** 8

    def workspace(self, dcut, method="hotrg"):
        return dcut ** 9

    def step_flops(self, dcut, method="hotrg"):
        return 2.0 * dcut ** 15

    def new_lane(self, dcut):
        return {"dcut": dcut}

    def create(self, req, stream, donor=None):
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        h = FakeHandle(req)
        h.ws = donor.ws if donor is not None else id(h)
        self.workspaces[h.ws] = self.workspaces.get(h.ws, 0) + 1
        self.max_workspaces = max(self.max_workspaces, len(self.workspaces))
        return h

    def dims(self, h):
        return tuple(h.dims)

    def step(self, handles, axis, dcut, method="hotrg"):
        self.calls.append((len(handles), axis, dcut, method))
        for h in handles:
            for a in range(4):
                if a != axis:
                    h.dims[a] = min(h.dims[a] ** 2, dcut)
            h.steps += 1

    def mark(self, stream):
        return {"polls": self.lag}

    def ready(self, ev):
        if ev is None:
            return True
        ev["polls"] -= 1
        return ev["polls"] <= 0

    def result(self, h):
        return float(h.req["beta"]) + h.steps

    def close(self, h):
        self.live -= 1
        self.workspaces[h.ws] -= 1
        if self.workspaces[h.ws] == 0:
            del self.workspaces[h.ws]



def test_every_request_completes_and_budget_is_respected():
    reqs = serving_requests(40, rate=2000.0, seed=1, dcuts=(4, 6, 8), kmin=2, kmax=4)
    be = FakeBackend()
    budget = 3 * 10 * 8 ** 8 + 8 ** 9
    srv = Server(be, budget)
    out = srv.serve(reqs, idle_sleep=0)
    assert out["completed"] == 40 and out["censored_active"] == 0
    assert srv.peak_used <= budget
    assert be.live == 0 and not be.workspaces and srv.used == 0
    # at most one workspace pool per lane (Dcut) at any time
    assert be.max_workspaces <= 3
    for r in srv.results:
        assert r["latency"] >= 0 and r["admitted"] >= r["arrival"] and r["done"] >= r["admitted"]
        # each run took exactly d * log2 L steps
        assert r["lnz"] == pytest.approx(r["beta"] + 4 * (r["L"].bit_length() - 1))


def test_same_shape_runs_share_calls():
    reqs = [{"id": i, "arrival": 0.0, "beta": 0.149 + 1e-4 * i, "h": 0.0, "dcut": 6, "L": 16, "method": "hotrg"}
            for i in range(5)]
    be = FakeBackend(lag=1)
    srv = Server(be, 10 ** 12)
    srv.serve(reqs, idle_sleep=0)
    assert all(n == 5 for n, _, _, _ in be.calls)
    assert len(be.calls) == 16


def test_continuous_admission_while_others_run():
    """A request that arrives while another is being stepped is admitted
    before that one finishes (no waiting for a full batch to drain)."""
    reqs = [{"id": 0, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 6, "L": 1024, "method": "hotrg"},
            {"id": 1, "arrival": 0.01, "beta": 0.150, "h": 0.0, "dcut": 6, "L": 16, "method": "hotrg"}]
    be = FakeBackend(lag=200)
    srv = Server(be, 10 ** 12)
    srv.serve(reqs, idle_sleep=1e-4)
    res = {r["id"]: r for r in srv.results}
    assert res[1]["admitted"] < res[0]["done"]
    assert res[1]["done"] < res[0]["done"]


def test_memory_bound_admission_waits_for_frees():
    reqs = [{"id": i, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 6, "L": 4, "method": "hotrg"} for i in range(3)]
    be = FakeBackend(lag=1)
    srv = Server(be, 10 * 6 ** 8 + 6 ** 9)   # room for one run at a time
    srv.serve(reqs, idle_sleep=0)
    assert be.max_live == 1 and len(srv.results) == 3
    done = sorted(srv.results, key=lambda r: r["id"])
    assert done[0]["done"] <= done[1]["admitted"] + 1e-9


def test_oversized_request_is_rejected():
    be = FakeBackend()
    srv = Server(be, 100)
    with pytest.raises(ValueError):
        srv.serve([{"id": 0, "arrival": 0.0, "beta": 0.15, "h": 0.0, "dcut": 8, "L": 4, "method": "hotrg"}])


def test_window_censors_unfinished_runs():
    reqs = [{"id": 0, "arrival": 0.0, "beta": 0.15, "h": 0.0, "dcut": 6, "L": 1024, "method": "hotrg"}]
    be = FakeBackend(lag=10 ** 9)
    srv = Server(be, 10 ** 12)
    out = srv.serve(reqs, window=0.05)
    assert out["completed"] == 0 and out["censored_active"] == 1
    srv.close()
    assert be.live == 0


def test_runs_of_a_lane_share_one_workspace_pool():
    """A HOTRG lane's runs share one pool that holds a slot per run of the
    batched step: four runs need four residents and four workspace shares;
    with room for two shares, two run at a time.  ATRG runs, stepped one call
    after another, share a single share."""
    reqs = [{"id": i, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 6, "L": 16, "method": "hotrg"} for i in range(4)]
    be = FakeBackend(lag=1)
    budget = 4 * (10 * 6 ** 8 + 6 ** 9)
    srv = Server(be, budget)
    srv.serve(reqs, idle_sleep=0)
    assert be.max_live == 4 and be.max_workspaces == 1
    assert srv.peak_used == budget and srv.used == 0
    assert all(n == 4 for n, _, _, _ in be.calls)
    be = FakeBackend(lag=1)
    srv = Server(be, 2 * (10 * 6 ** 8 + 6 ** 9))
    srv.serve(reqs, idle_sleep=0)
    assert be.max_live == 2 and len(srv.results) == 4 and srv.used == 0
    at = [dict(r, method="atrg") for r in reqs]
    be = FakeBackend(lag=1)
    srv = Server(be, 4 * 10 * 6 ** 8 + 6 ** 9)   # four residents, one share
    srv.serve(at, idle_sleep=0)
    assert be.max_live == 4 and be.max_workspaces == 1 and srv.used == 0


def test_lane_cap_bounds_a_round_and_keeps_arrival_order():
    """Dcut 8 (7e13 flop per step) gets one run at a time under a 4e13 round;
    Dcut 4 requests behind them are not held back."""
    reqs = [{"id": i, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 8, "L": 4, "method": "hotrg"} for i in range(3)]
    reqs += [{"id": 3 + i, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 4, "L": 4, "method": "hotrg"}
             for i in range(3)]
    be = FakeBackend(lag=1)
    srv = Server(be, 10 ** 12)
    assert srv.lane_cap(8) == 1 and srv.lane_cap(4) == 256
    srv.serve(reqs, idle_sleep=0)
    res = {r["id"]: r for r in srv.results}
    assert len(res) == 6
    # the Dcut 8 runs ran one after another, in arrival order
    assert res[0]["done"] <= res[1]["admitted"] + 1e-9 and res[1]["done"] <= res[2]["admitted"] + 1e-9
    # the Dcut 4 runs were admitted at once, beside the first Dcut 8 run
    assert all(res[3 + i]["admitted"] < res[0]["done"] for i in range(3))
    # calls on the Dcut 8 lane step one run
    assert all(n == 1 for n, _, dc, _ in be.calls if dc == 8)


def test_methods_get_separate_lanes():
    """HOTRG and ATRG requests of one Dcut go to two lanes; both complete
    with d log2 L steps each, and no call mixes the methods."""
    reqs = [{"id": i, "arrival": 0.0, "beta": 0.149, "h": 0.0, "dcut": 6, "L": 16,
             "method": "atrg" if i % 2 else "hotrg"} for i in range(6)]
    be = FakeBackend()
    srv = Server(be, 10 ** 12)
    out = srv.serve(reqs, idle_sleep=0)
    assert out["completed"] == 6
    assert set(srv.lanes) == {("hotrg", 6), ("atrg", 6)}
    assert {r["method"] for r in srv.results} == {"hotrg", "atrg"}
    for r in srv.results:
        assert r["lnz"] == pytest.approx(r["beta"] + 16)
    assert {c[3] for c in be.calls} == {"hotrg", "atrg"}
