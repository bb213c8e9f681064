"""Start level of the sweep: potentials of the pairs (A at T_X level s0,
B at T_K level L - s0) summed directly over the sources in B (the plain
procedure of Section 2.1), then the butterfly from there.  The start level
is chosen by the plan (BFSFT_START_LEVEL unset) or forced; the oracle runs
the same sweep with the same start level.

Bars: FP64 vs the oracle O2 rel-l2 <= 1e-10; the reduced precisions within 3x
the deviation measured on an MI355X for the same case; the 1e-6 gate
on the c2 error subset against the direct sum.
"""
import numpy as np
import pytest

from conftest import rel_l2, within_measured
from paper_0801_1524_amd import synth

pytestmark = pytest.mark.gpu

EPS = {4: 0.05, 5: 6e-3, 7: 3e-4, 9: 1.5e-6}


@pytest.fixture(scope="module")
def bf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0801_1524_amd as bf
    bf.lib()
    return bf


def run(bf, P, precision, start, monkeypatch):
    if start is None:
        monkeypatch.delenv("BFSFT_START_LEVEL", raising=False)
    else:
        monkeypatch.setenv("BFSFT_START_LEVEL", str(start))
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, precision) as plan:
        u = plan.execute(P.f).cpu().numpy()
        s0 = plan.info()["start_level"]
    if start is not None:
        assert s0 == min(start, plan_levels(P))
    return u, s0


def plan_levels(P):
    return int(np.ceil(np.log2(P.N)))


def oracle_u(oracle_mod, P, s0, x=None):
    x = P.x if x is None else x
    return oracle_mod.Butterfly(P.d, P.N, P.p, x, P.k).run(P.f, start_level=s0)


@pytest.mark.parametrize("start", [None, 1, 2, 4, 6])
def test_c1_fp64_vs_oracle(bf, oracle_mod, monkeypatch, start):
    P = synth.config("c1")
    u, s0 = run(bf, P, "fp64", start, monkeypatch)
    assert rel_l2(u, oracle_u(oracle_mod, P, s0)) <= 1e-10
    S = synth.error_subset(P.nx, 1)
    assert rel_l2(u[S], oracle_mod.direct(P.x, P.k, P.f, P.N, S)) <= EPS[P.p]


def test_auto_start_is_above_the_leaves_at_one_sample_per_unit(bf, monkeypatch):
    # 1 source per unit length: leaves hold about one source, far fewer than p^2
    _, s0 = run(bf, synth.config("c1"), "fp64", None, monkeypatch)
    assert s0 >= 1


# rel-l2 vs O2 at the same start level, measured on an MI355X (the bar is 3x)
MEASURED_C1_S3 = {"mixed": 1.5e-7, "fp32": 3.78e-7, "fp16x2": 4.38e-7, "bf16x3": 2.01e-7}
# (the largest over the seven transforms)
MEASURED_BATCH_S2 = {"mixed": 1.53e-7, "bf16x3": 2.89e-7}


@pytest.mark.parametrize("precision", ["mixed", "fp32", "fp16x2", "bf16x3"])
def test_c1_lower_precisions(bf, oracle_mod, monkeypatch, precision):
    P = synth.config("c1")
    u, s0 = run(bf, P, precision, 3, monkeypatch)
    within_measured(rel_l2(u, oracle_u(oracle_mod, P, s0)), MEASURED_C1_S3[precision], f"c1 start 3 {precision}")


@pytest.mark.parametrize("N,p,start", [(1000, 7, 2), (3001, 9, 3), (512, 5, 9)])
def test_non_power_of_two_and_full_direct(bf, oracle_mod, monkeypatch, N, p, start):
    P = synth.curve_problem(N, p, seed=N + start)
    u, s0 = run(bf, P, "fp64", start, monkeypatch)
    assert rel_l2(u, oracle_u(oracle_mod, P, s0)) <= 1e-10


@pytest.mark.parametrize("start", [1, 2, 4])
def test_3d(bf, oracle_mod, monkeypatch, start):
    N = 16
    x = synth.sphere(N)
    k = synth.sphere(N, radius=0.3)
    P = synth.Problem("s3", 3, N, 4, x, k, synth.gaussian_sources(len(k), 3))
    u, s0 = run(bf, P, "fp64", start, monkeypatch)
    assert rel_l2(u, oracle_u(oracle_mod, P, s0)) <= 1e-10


def test_potentials_at_and_below_the_start(bf, oracle_mod, monkeypatch):
    P = synth.config("c1")
    s0 = 3
    monkeypatch.setenv("BFSFT_START_LEVEL", str(s0))
    ob = oracle_mod.Butterfly(P.d, P.N, P.p, P.x, P.k)
    L = ob.L
    for lvl in (L - s0, L - s0 - 2):
        _, du, _ = ob.run(P.f, dump_level=lvl, start_level=s0)
        with bf.Plan(P.d, P.N, P.p, P.x, P.k, "fp64") as plan:
            _, pot = plan.execute_probe(P.f, lvl)
            pot = pot.cpu().numpy()
            gx, gk = plan.boxes("x", L - lvl), plan.boxes("k", lvl)
            with pytest.raises(Exception):
                plan.execute_probe(P.f, L - s0 + 1)  # no potentials above the start
        ox, ok = ob.boxes("x", L - lvl), ob.boxes("k", lvl)
        ix = {tuple(r): i for i, r in enumerate(ox)}
        ik = {tuple(r): i for i, r in enumerate(ok)}
        ref = du[np.array([ix[tuple(r)] for r in gx])][:, np.array([ik[tuple(r)] for r in gk])]
        assert rel_l2(pot, ref) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_full_size_auto_start(bf, oracle_mod, monkeypatch, precision):
    """N = 65536, p = 9 with the plan's own start level: the 1e-6 gate, and
    (FP64) the oracle with the same start level restricted to 24 targets."""
    c2 = synth.config("c2")
    u, s0 = run(bf, c2, precision, None, monkeypatch)
    S = synth.error_subset(c2.nx, 2)
    err = rel_l2(u[S], oracle_mod.direct(c2.x, c2.k, c2.f, c2.N, S))
    assert err <= 1e-6, err
    if precision == "fp64":
        T = np.sort(np.random.default_rng(17).choice(c2.nx, 24, replace=False))
        assert rel_l2(u[T], oracle_u(oracle_mod, c2, s0, x=c2.x[T])) <= 1e-10


def test_adjoint_auto_start_vs_direct(bf, oracle_mod, monkeypatch):
    monkeypatch.delenv("BFSFT_START_LEVEL", raising=False)
    P = synth.config("c1")
    g = synth.gaussian_sources(P.nx, 77)
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, "fp64") as plan:
        v = plan.execute_adjoint(g).cpu().numpy()
    S = np.arange(0, P.nk, 7)
    vd = np.conj(oracle_mod.direct(P.k, P.x, np.conj(g), P.N, S))
    assert rel_l2(v[S], vd) <= EPS[P.p]


# ------------------------------------------------------------------ batched

def _batch(count=7, seed=11):
    return synth.batched_config(count=count, p=7, nmin=48, nmax=1500, seed=seed)


def _split(u, probs):
    out, o = [], 0
    for q in probs:
        out.append(u[o:o + q.nx])
        o += q.nx
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed", "bf16x3"])
def test_batched_forced_start_vs_serial_and_oracle(bf, oracle_mod, monkeypatch, precision):
    """Every transform starts 2 levels above its leaves: the batched graph
    (a direct-sum launch for all transforms, then the steps) equals the same
    transforms run one by one, and each equals the oracle with start 2."""
    monkeypatch.setenv("BFSFT_START_LEVEL", "2")
    probs = _batch()
    B = bf.BatchedPlan([(q.N, q.x, q.k) for q in probs], 2, 7, precision)
    f = np.concatenate([q.f for q in probs])
    ug = B.execute(f).cpu().numpy()
    us = B.execute(f, serial=True).cpu().numpy()
    B.close()
    assert rel_l2(ug, us) <= 1e-14
    for q, u in zip(probs, _split(ug, probs)):
        ub = oracle_mod.Butterfly(2, q.N, q.p, q.x, q.k).run(q.f, start_level=2)
        if precision == "fp64":
            assert rel_l2(u, ub) <= 1e-10, (q.name, q.N)
        else:
            within_measured(rel_l2(u, ub), MEASURED_BATCH_S2[precision], f"batched start 2 {precision} {q.name}")


def test_batched_auto_start_vs_serial_and_direct(bf, oracle_mod, monkeypatch):
    """Each transform with its own chosen start level (the 1-per-unit-length
    curves start above the leaves): graph equals serial, outputs within the
    method's accuracy of the direct sum."""
    monkeypatch.delenv("BFSFT_START_LEVEL", raising=False)
    probs = _batch(count=9, seed=4)
    B = bf.BatchedPlan([(q.N, q.x, q.k) for q in probs], 2, 7, "fp64")
    f = np.concatenate([q.f for q in probs])
    ug = B.execute(f).cpu().numpy()
    us = B.execute(f, serial=True).cpu().numpy()
    B.close()
    assert rel_l2(ug, us) <= 1e-14
    for q, u in zip(probs, _split(ug, probs)):
        assert rel_l2(u, oracle_mod.direct(q.x, q.k, q.f, q.N)) <= EPS[7], (q.name, q.N)


@pytest.mark.parametrize("d,N,p,n,precision,start", [
    (2, 1 << 24, 7, 1000, "fp64", 0), (2, 1 << 24, 7, 1000, "fp64", None),
    (2, 1 << 24, 7, 1000, "mixed", None), (3, 1 << 16, 5, 400, "fp64", 0),
    (3, 1 << 16, 5, 400, "fp64", None)])
def test_largest_N(bf, oracle_mod, monkeypatch, d, N, p, n, precision, start):
    """The largest frequency bound a plan accepts (2^24 in 2D, 2^16 in 3D:
    24 and 16 levels), with a few hundred points per side at random on
    closed curves and spheres: every output against the direct sum at the
    method's accuracy, and at FP64 sampled targets against the oracle
    butterfly at the same start level (exactly their ancestor pairs)."""
    P = synth.sparse_problem(d, N, p, n, seed=N + p)
    u, s0 = run(bf, P, precision, start, monkeypatch)
    assert rel_l2(u, oracle_mod.direct(P.x, P.k, P.f, P.N)) <= EPS[p]
    if precision == "fp64":
        T = np.arange(0, P.nx, 40 if d == 2 else 25)
        assert rel_l2(u[T], oracle_u(oracle_mod, P, s0, x=P.x[T])) <= 1e-10


@pytest.mark.parametrize("start", ["chosen", "0", "12"])
def test_timing_intervals(bf, monkeypatch, start):
    """The per-launch event intervals (what bench.py reports per level):
    positive for the translated levels below the start, zero for the levels
    above it (which record no event), positive for the start and the final
    evaluation; C1 has 12 levels, so start 12 translates nothing."""
    if start == "chosen":
        monkeypatch.delenv("BFSFT_START_LEVEL", raising=False)
    else:
        monkeypatch.setenv("BFSFT_START_LEVEL", start)
    P = synth.config("c1")
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, "mixed") as plan:
        plan.timing_begin(3)
        for _ in range(3):
            plan.execute(P.f)
        tm = plan.timing_end()
        inf = plan.info()
    L, s0 = inf["levels"], inf["start_level"]
    if start != "chosen":
        assert s0 == int(start)
    assert tm["executes"] == 3
    assert tm["leaf_ms"] > 0 and tm["final_ms"] > 0
    for l in range(L):
        if l < L - s0:
            assert tm["translate_ms"][l] > 0, l
        else:
            assert tm["translate_ms"][l] == 0, l
