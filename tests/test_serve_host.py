"""The simulation server's host logic on the CPU, over a stand-in of the
library binding built on the oracle (tests/fake_capi.py): admission by the
memory budget (first in, first out), batched ticks, retirement on
convergence and at the step cap, rejection of a request that can never
fit and of an unphysical one, isolation of a request that goes
non-finite mid-run, and the statistics over the finished requests."""
import numpy as np

from inputs import components as C
from inputs import fields as Fi
from tests import fake_capi
from tests import workloads as W


class _PoisonAfterFirstTick(fake_capi.Simulation):
    """A simulation whose populations turn non-finite after its first
    batched step (the fault the library reports as a sticky ENONFINITE)."""
    poison_shape = (24, 4)

    def run(self, nsteps):
        rc = super().run(nsteps)
        if rc == 0 and (self.o.nx, self.o.ny) == self.poison_shape:
            self.poke(0, 1, 5, float("nan"))
        return rc


def test_server_admission_retirement_and_isolation(monkeypatch):
    from paper_2306_10652_amd import serve
    fake = fake_capi
    monkeypatch.setattr(fake, "Simulation", _PoisonAfterFirstTick)
    monkeypatch.setattr(serve, "capi", fake)
    S = W.states()

    def comps(case):
        return C.table_ii_components(case)[:2]

    reqs = []
    c2, T2 = comps(2)
    c3, T3 = comps(3)
    v2, v3 = S["vle2"], S["vle3"]
    # 0: a uniform vapour, a fixed point: converges on its first tick
    reqs.append(serve.Request(0, c2, T2, fake.D2Q9, (16, 4), Fi.uniform(16, 4, v2["rho_V"])))
    # 1, 2: slabs that do not settle within the step cap
    reqs.append(serve.Request(1, c2, T2, fake.D2Q9, (32, 4), Fi.slab(32, 4, v2["rho_V"], v2["rho_L"], 0.5)))
    reqs.append(serve.Request(2, c3, T3, fake.D2Q9, (32, 4), Fi.slab(32, 4, v3["rho_V"], v3["rho_L"], 0.5)))
    # 3: larger than the whole budget
    reqs.append(serve.Request(3, c2, T2, fake.D2Q9, (4096, 4096), Fi.uniform(4, 4, v2["rho_V"])))
    # 4: an unphysical field (a zero density)
    bad = Fi.uniform(16, 4, v2["rho_V"])
    bad[0, 0, 0, 0] = 0.0
    reqs.append(serve.Request(4, c2, T2, fake.D2Q9, (16, 4), bad))
    # 5: goes non-finite after its first tick
    reqs.append(serve.Request(5, c3, T3, fake.D2Q9, (24, 4), Fi.slab(24, 4, v3["rho_V"], v3["rho_L"], 0.5)))
    for r in reqs:
        r.precision = fake.FP64
        r.tol = 1e-12
        r.max_steps = 1000
    sizes = [r.nbytes() for r in reqs]
    # room for the two largest small requests at a time, not for all of them
    budget = sizes[1] + sizes[2]
    srv = serve.Server(budget, chunk=200, stream=object(), streams=1, keep_fields=True)
    peak = []
    admit = srv._admit

    def admit_and_check(req, now):
        slot = admit(req, now)
        peak.append(srv.used)
        return slot
    srv._admit = admit_and_check
    done = {r.rid: r for r in srv.run(reqs)}

    assert sorted(done) == list(range(6))
    assert max(peak) <= budget and srv.used == 0
    # first in, first out: 2 waits for 0 to retire, 5 for 1
    assert done[1].admit_t <= done[0].finish_t <= done[2].admit_t
    assert done[5].admit_t >= done[1].finish_t
    assert done[0].status == 0 and done[0].converged and done[0].steps == 200
    for k in (1, 2):
        r = done[k]
        assert r.status == 0 and not r.converged and r.steps == 1000
        # the served state is the state of the same request stepped alone
        m = fake.Mixture.from_components(r.comps, r.T)
        alone = fake.Simulation(m, r.lattice, r.precision, r.shape, r.rho)
        alone.run(r.steps)
        assert np.array_equal(r.result["populations"], alone.read_populations())
    assert done[3].status == -1 and done[3].admit_t is None
    assert done[4].status == fake.EUNPHYSICAL
    assert done[5].status == fake.ENONFINITE and done[5].steps == 200
    st = serve.latency_stats(list(done.values()))
    assert (st["requests"], st["converged"], st["capped"], st["failed"]) == (6, 1, 2, 3)
    assert st["steps_max"] == 200
