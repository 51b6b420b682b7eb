"""HIP-graph replay of the multi-shift CG loop: the same kernels in the same order as the
eager launches, so every replay must reproduce the eager result bit for bit.

Each case computes eager references with graphs off, then turns graphs on and calls the
solver repeatedly (first call captures, later calls replay from the cache), with unrelated
eager device work and synchronisations between the calls, checking every call.
"""

import numpy as np
import pytest

import paper_1701_00726_amd as bri
import synth
from tests._gpu import field, need_gpu, torch

pytestmark = pytest.mark.gpu


def _eager_noise():
    a = torch.randn(512, 512, device="cuda", dtype=torch.float64)
    (a @ a).sum().item()
    torch.cuda.synchronize()


@pytest.fixture(autouse=True)
def _graphs_back_on():
    yield
    if torch.cuda.is_available():
        bri.set_solver_graphs(True)


@pytest.mark.parametrize("L,inner,nrhs", [((4, 4, 4, 4), bri.F64, 1), ((8, 8, 8, 8), bri.F64, 3),
                                          ((8, 8, 8, 8), bri.F32, 2), ((4, 4, 4, 8), bri.F32_BF16W, 1)])
def test_graph_replay_matches_eager(L, inner, nrhs):
    need_gpu()
    U, _ = field(L, "cfg1", 1)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L, Ud, bri.F64, tbc=1)
    Wlo = None if inner == bri.F64 else bri.build_links(L, Ud, inner, tbc=1)
    op = bri.OverlapOp(L, W, kl_n=12, tol=1e-12, tbc=1, Wlo=Wlo, inner=inner, nrhs=nrhs)
    srcs = [bri.spinor_to_device(synth.gaussian_source(L, 900 + i, nrhs=nrhs)) for i in range(3)]
    bri.set_solver_graphs(False)
    ref = [op.apply(b)[0].clone() for b in srcs]
    refs = [op.sign(b)[0].clone() for b in srcs]
    bri.set_solver_graphs(True)
    for rep in range(3):
        for i, b in enumerate(srcs):
            _eager_noise()
            out, st = op.apply(b)
            assert torch.equal(out, ref[i]), (rep, i, st.iters)
            assert torch.equal(op.sign(b)[0], refs[i]), (rep, i)


def test_graph_with_iteration_cap_not_a_multiple_of_the_block():
    need_gpu()
    L = (8, 8, 8, 8)
    U, _ = field(L, "cfg2", 0)
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    b = bri.spinor_to_device(synth.gaussian_source(L, 77))
    op = bri.OverlapOp(L, W, kl_n=8, tol=1e-14, max_iter=13)
    bri.set_solver_graphs(False)
    ref, st0 = op.apply(b, allow_noconv=True)
    ref = ref.clone()
    bri.set_solver_graphs(True)
    for _ in range(2):
        out, st = op.apply(b, allow_noconv=True)
        assert st.status == st0.status == bri.ENOCONV and st.iters == st0.iters == 13
        assert torch.equal(out, ref)


def test_graph_gradient_matches_eager():
    need_gpu()
    L = (4, 4, 4, 4)
    U, _ = field(L, "rough", 0)
    Ud = bri.links_to_device(U)
    W = bri.build_links(L, Ud, bri.F64)
    rng = np.random.default_rng(3)
    chi = bri.spinor_to_device(rng.standard_normal((1, 256, 4, 3)) + 1j * rng.standard_normal((1, 256, 4, 3)))[0]
    psi = bri.spinor_to_device(rng.standard_normal((1, 256, 4, 3)) + 1j * rng.standard_normal((1, 256, 4, 3)))[0]
    op = bri.OverlapOp(L, W, kl_n=6)
    bri.set_solver_graphs(False)
    F0, _, g0, _ = op.grad(Ud, chi, psi)
    F0, g0 = F0.clone(), g0.clone()
    bri.set_solver_graphs(True)
    for _ in range(3):
        _eager_noise()
        F, _, g, _ = op.grad(Ud, chi, psi)
        assert torch.equal(F, F0) and torch.equal(g, g0)


def test_graph_cache_eviction_and_concurrent_threads():
    """More solve layouts than the graph cache holds (every operator has its own workspace, so
    its own graphs): evicted graphs are captured again and give the same bits; then two host
    threads apply their operators at once on their own streams (graphs are looked up, captured
    and launched under the cache lock), every result bit for bit the eager one."""
    import threading

    need_gpu()
    L = (4, 4, 4, 4)
    U, _ = field(L, "cfg1")
    W = bri.build_links(L, bri.links_to_device(U), bri.F64)
    b = bri.spinor_to_device(synth.gaussian_source(L, synth.SOURCE_SEED_BASE + 9))
    bri.set_solver_graphs(False)
    ref, _ = bri.OverlapOp(L, W, kl_n=8, tol=1e-12).apply(b)
    bri.set_solver_graphs(True)
    ops = [bri.OverlapOp(L, W, kl_n=8, tol=1e-12) for _ in range(20)]
    for op in ops + ops[::-1]:
        out, _ = op.apply(b)
        assert torch.equal(out, ref)
        _eager_noise()
    errors = []

    def work(op, stream):
        try:
            with torch.cuda.stream(stream):
                for _ in range(6):
                    out, _ = op.apply(b, stream=stream)
                    stream.synchronize()
                    if not torch.equal(out, ref):
                        errors.append("mismatch")
        except Exception as e:  # reported below, the thread must not die silently
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(ops[i], torch.cuda.Stream())) for i in (0, 17)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors


def test_eviction_while_another_thread_runs_its_graphs():
    """One host thread keeps applying an operator on a larger lattice (its graphs in flight on
    its stream) while a second thread cycles through more solve layouts than the cache holds,
    so cache entries are evicted while graphs of the first thread may still run; eviction waits
    for each entry's last launch.  Every result bit for bit the eager one."""
    import threading

    need_gpu()
    Lb, Ls = (8, 8, 8, 8), (4, 4, 4, 4)
    Ub, _ = field(Lb, "cfg1")
    Us, _ = field(Ls, "cfg1")
    Wb = bri.build_links(Lb, bri.links_to_device(Ub), bri.F64)
    Ws = bri.build_links(Ls, bri.links_to_device(Us), bri.F64)
    bb = bri.spinor_to_device(synth.gaussian_source(Lb, synth.SOURCE_SEED_BASE + 11))
    bs = bri.spinor_to_device(synth.gaussian_source(Ls, synth.SOURCE_SEED_BASE + 12))
    bri.set_solver_graphs(False)
    refb, _ = bri.OverlapOp(Lb, Wb, kl_n=16, tol=1e-12).apply(bb)
    refs, _ = bri.OverlapOp(Ls, Ws, kl_n=8, tol=1e-12).apply(bs)
    bri.set_solver_graphs(True)
    big = bri.OverlapOp(Lb, Wb, kl_n=16, tol=1e-12)
    smalls = [bri.OverlapOp(Ls, Ws, kl_n=8, tol=1e-12) for _ in range(24)]
    errors, stop = [], threading.Event()

    def runner():
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                while not stop.is_set():
                    out, _ = big.apply(bb, stream=s)
                    s.synchronize()
                    if not torch.equal(out, refb):
                        errors.append("big mismatch")
        except Exception as e:  # reported below
            errors.append(repr(e))

    def evictor():
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                for _ in range(3):
                    for op in smalls:  # 24 layouts x 2 block lengths > 16 cache entries
                        out, _ = op.apply(bs, stream=s)
                        s.synchronize()
                        if not torch.equal(out, refs):
                            errors.append("small mismatch")
        except Exception as e:  # reported below
            errors.append(repr(e))
        finally:
            stop.set()

    threads = [threading.Thread(target=runner), threading.Thread(target=evictor)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=180)
    stop.set()
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors[:5]
