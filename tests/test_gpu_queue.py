"""Job-queue launches on the GPU: the independent small jobs of one call that
share a shape class run as one launch per pass over all of them.

Checks: the queue kernels actually ran (their profile entries), every job of
the call is bit-identical to the same job run alone (an eligible job always
runs through the queue kernels) and equal to rounding to the per-job
kernels (the queue switched off: relative L2 <= 1e-6 for complex64, 1e-14
for complex128; the two compile the same passes with different constant
folding, which may fuse a multiply-add differently); FP64-oracle parity for
one job of each class (complex64 relative L2 <= 2e-5, complex128 <= 1e-12);
jobs with elements or a dependency on another job of the call keep call
order; a captured HIP graph of the queue path replays equal to eager runs."""
import os

import numpy as np
import pytest

import oracle
from tests._util import announce, crandn, rel, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {np.complex64: 2e-5, np.complex128: 1e-12}
ROUNDING = {np.complex64: 1e-6, np.complex128: 1e-14}


def _close(a, b, bar):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) <= bar


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def _jobs(rng, count, dtype):
    """Small jobs over a few classes: square and ragged grids (the ragged
    ones fill less than half of their padded extent), batches of 1 to 3,
    ASM, Fresnel and direct integration, random wavelength and distance."""
    tp = _tp()
    shapes = [(64, 64), (100, 100), (128, 128), (200, 256), (256, 256), (512, 512), (37, 64)]
    methods = ["asm", "asm", "fresnel", "di"]
    out = []
    for k in range(count):
        ny, nx = shapes[k % len(shapes)]
        meth = methods[(k // len(shapes)) % len(methods)]
        d = float(rng.uniform(3e-6, 12e-6))
        lam = float(rng.uniform(420e-9, 780e-9))
        z = float(rng.uniform(2e-3, 8e-2))
        u = crandn(rng, 1 + k % 3, ny, nx, dtype=dtype)
        g = crandn(rng, 1 + k % 3, ny, nx, dtype=dtype)
        out.append(dict(u=u, g=g, opt=tp.Optics(dy=d, dx=d, wavelength=lam, z=z, method=meth, pad=2), meth=meth))
    return out


def _profiled(fn):
    from paper_2411_18591_amd import _capi
    torch.cuda.synchronize()
    _capi.profile_begin()
    res = fn()
    torch.cuda.synchronize()
    return res, _capi.profile_end()


def _no_queue(fn):
    os.environ["TOPROP_NO_QUEUE"] = "1"
    try:
        res = fn()
        torch.cuda.synchronize()
    finally:
        del os.environ["TOPROP_NO_QUEUE"]
    return res


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_queue_groups_equal_solo_runs_and_oracle(dtype):
    tp = _tp()
    rng = np.random.default_rng(4401 if dtype == np.complex64 else 4402)
    jobs = _jobs(rng, 28 if dtype == np.complex64 else 14, dtype)
    announce(f"queue: {len(jobs)} small jobs, {np.dtype(dtype).name}, forward + backward calls")
    us = [to_gpu(j["u"], torch) for j in jobs]
    gs = [to_gpu(j["g"], torch) for j in jobs]
    opts = [j["opt"] for j in jobs]

    def both():
        return tp.propagate_jobs(us, opts), tp.propagate_backward_jobs(gs, opts)

    (outs, gins), prof = _profiled(both)
    names = " ".join(prof)
    for p in ("fwd.queue_row_fwd", "fwd.queue_col", "fwd.queue_row_inv", "bwd.queue_row_fwd",
              "bwd.queue_col", "bwd.queue_row_inv"):
        assert p in names, f"no {p} launch: {sorted(prof)}"
    # at most half the launches of the per-job passes (three per job and direction)
    assert sum(n for k, (n, _) in prof.items() if "queue" in k) <= 3 * len(jobs)
    outs_nq, gins_nq = _no_queue(both)
    seen = set()
    for k, (j, u, g, o, gi, o2, gi2) in enumerate(zip(jobs, us, gs, outs, gins, outs_nq, gins_nq)):
        so = tp.propagate(u, j["opt"])
        sg = tp.propagate_backward(g, j["opt"])
        torch.cuda.synchronize()
        assert torch.equal(o, so), f"job {k} forward differs from its solo run"
        assert torch.equal(gi, sg), f"job {k} backward differs from its solo run"
        assert _close(o, o2, ROUNDING[dtype]) and _close(gi, gi2, ROUNDING[dtype]), \
            f"job {k} differs from the call without the queue beyond rounding"
        cls = (j["u"].shape[-2:], j["meth"])
        if cls in seen:
            continue
        seen.add(cls)
        meth = {"asm": oracle.ASM, "fresnel": oracle.FRESNEL, "di": oracle.DI}[j["meth"]]
        op = j["opt"]
        announce(f"queue: oracle parity job {k} {cls}")
        pad = op.padded_shape(*j["u"].shape[-2:])
        exp = oracle.propagate(j["u"].astype(np.complex128), op.dy, op.dx, op.wavelength, op.z, meth, 2,
                               padded=pad)
        assert rel(to_np(o), exp) <= TOL[dtype], (k, cls)
        expg = oracle.propagate(j["g"].astype(np.complex128), op.dy, op.dx, op.wavelength, op.z, meth, 2,
                                adjoint=True, padded=pad)
        assert rel(to_np(gi), expg) <= TOL[dtype], (k, cls)


def test_queue_leaves_out_elements_and_dependent_jobs():
    """Eligible jobs mixed with a phase-mask job and a job that reads another
    job's output: results equal the jobs run one by one in call order, and
    the call with the queue switched off to rounding."""
    tp = _tp()
    rng = np.random.default_rng(4403)
    announce("queue: mixed eligible and ineligible jobs")
    n = 64
    opt = tp.Optics(dy=6e-6, dx=6e-6, wavelength=633e-9, z=0.01, pad=2)
    us = [to_gpu(crandn(rng, 1, n, n, dtype=np.complex64), torch) for _ in range(6)]
    outs = [torch.empty_like(u) for u in us]
    phi = to_gpu((rng.random((n, n)) * 2 * np.pi).astype(np.float32), torch)
    els = [{} for _ in us]
    els[2] = {"phase": phi}
    # job 4 reads job 1's output (same call): it must run after job 1
    fields = list(us)
    fields[4] = outs[1]

    def call():
        return tp.propagate_jobs(fields, [opt] * len(us), outs=outs, elements=els)

    _, prof = _profiled(call)
    got = [o.clone() for o in outs]
    assert any("queue" in k for k in prof), sorted(prof)
    ref = []
    for k in range(len(us)):
        src = ref[1] if k == 4 else us[k]
        ref.append(tp.propagate(src, opt, **els[k]))
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(got, ref)):
        assert torch.equal(a, b), f"job {k} differs from the one-by-one run"
    _no_queue(call)
    for k, (a, b) in enumerate(zip(got, outs)):
        assert _close(a, b, ROUNDING[np.complex64]), f"job {k} differs from the call without the queue"


def test_queue_graph_capture_replays_match_eager():
    """Forward + backward over 12 small jobs captured into one HIP graph;
    three replays with new inputs copied in, each against an eager run."""
    tp = _tp()
    announce("queue: hipGraph capture of job-queue forward+backward")
    rng = np.random.default_rng(4404)
    shapes = [(64, 64), (128, 128), (256, 256)] * 4
    opts = [tp.Optics(dy=5e-6, dx=5e-6, wavelength=500e-9 + 20e-9 * k, z=0.004 + 0.003 * k, pad=2)
            for k in range(len(shapes))]
    fields = [torch.zeros((1 + k % 2,) + s, dtype=torch.complex64, device="cuda") for k, s in enumerate(shapes)]
    gouts = [torch.zeros_like(f) for f in fields]
    outs = [torch.empty_like(f) for f in fields]
    gins = [torch.empty_like(f) for f in fields]

    def step():
        tp.propagate_jobs(fields, opts, outs=outs)
        tp.propagate_backward_jobs(gouts, opts, grad_ins=gins)

    def fill(seed):
        r = np.random.default_rng(seed)
        for f, g in zip(fields, gouts):
            f.copy_(to_gpu(crandn(r, *f.shape, dtype=np.complex64), torch))
            g.copy_(to_gpu(crandn(r, *g.shape, dtype=np.complex64), torch))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fill(1)
        step()  # sizes the workspaces outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        fill(200 + rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in outs + gins]
        junk = tp.propagate(to_gpu(crandn(rng, 1, 48, 48, dtype=np.complex64), torch), opts[0])  # eager work
        step()
        torch.cuda.synchronize()
        for a, b in zip(got, outs + gins):
            assert torch.equal(a, b), f"replay {rep} differs from eager"
        del junk
