"""Calls captured into HIP graphs owned by the library (to_graph_create /
to_graph_launch / to_graph_destroy).

Checks: a forward call and an adjoint call over jobs of several shapes
(job-queue classes, a per-job 1024^2 job, a phase-mask job with its mask
gradient, a ragged grid) are captured after running once; three replays
with new inputs copied in, with eager work in between, equal eager calls
bit for bit; a workspace that grows while the graphs are alive (a larger
eager call) does not invalidate them; releasing the workspaces is refused
while a graph is alive and allowed after the graphs are destroyed."""
import numpy as np
import pytest

from tests._util import announce, crandn, to_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tp():
    import paper_2411_18591_amd as tp
    return tp


def test_library_graphs_replay_like_eager_calls():
    tp = _tp()
    from paper_2411_18591_amd import _capi
    announce("graph: library-owned capture of a forward and an adjoint call")
    rng = np.random.default_rng(6101)
    shapes = [(64, 64), (64, 64), (128, 128), (256, 256), (256, 256), (100, 100), (37, 64), (1024, 1024),
              (512, 512), (128, 128)]
    opts = [tp.Optics(dy=6e-6, dx=6e-6, wavelength=480e-9 + 25e-9 * k, z=0.005 + 0.004 * k, pad=2)
            for k in range(len(shapes))]
    fields = [torch.zeros((1 + k % 2,) + s, dtype=torch.complex64, device="cuda") for k, s in enumerate(shapes)]
    gouts = [torch.zeros_like(f) for f in fields]
    outs = [torch.empty_like(f) for f in fields]
    gins = [torch.empty_like(f) for f in fields]
    phi = to_gpu((rng.random(shapes[2]) * 2 * np.pi).astype(np.float32), torch)
    gphi = torch.zeros_like(phi)
    els = [{} for _ in shapes]
    els[2] = {"phase": phi}
    gphs = [None] * len(shapes)
    gphs[2] = gphi

    def fill(seed):
        r = np.random.default_rng(seed)
        for f, g in zip(fields, gouts):
            f.copy_(to_gpu(crandn(r, *f.shape, dtype=np.complex64), torch))
            g.copy_(to_gpu(crandn(r, *g.shape, dtype=np.complex64), torch))
        gphi.zero_()

    def eager():
        gphi.zero_()
        tp.propagate_jobs(fields, opts, outs=outs, elements=els)
        tp.propagate_backward_jobs(gouts, opts, saved_ins=fields, grad_ins=gins, grad_phases=gphs, elements=els)

    fill(1)
    _, gf = tp.propagate_jobs(fields, opts, outs=outs, elements=els, graph=True)
    _, gb = tp.propagate_backward_jobs(gouts, opts, saved_ins=fields, grad_ins=gins, grad_phases=gphs,
                                       elements=els, graph=True)
    torch.cuda.synchronize()
    for rep in range(3):
        fill(300 + rep)
        if rep == 1:
            # a larger eager call grows the workspaces while the graphs live
            big = to_gpu(crandn(rng, 2, 2048, 2048, dtype=np.complex64), torch)
            tp.propagate(big, tp.Optics(dy=4e-6, dx=4e-6, wavelength=600e-9, z=0.02, pad=2))
            del big
        torch.cuda.synchronize()
        gf.launch()
        gb.launch()
        torch.cuda.synchronize()
        got = [t.clone() for t in outs + gins + [gphi]]
        junk = tp.propagate(to_gpu(crandn(rng, 1, 48, 48, dtype=np.complex64), torch), opts[0])  # eager work
        eager()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(got, outs + gins + [gphi])):
            assert torch.equal(a, b), f"replay {rep}: tensor {k} differs from the eager call"
        del junk
    with pytest.raises(_capi.ToError) as e:
        _capi.lib()  # noqa: B018
        _capi.check(_capi.lib().to_release())
    assert e.value.status == _capi.TO_E_INVAL
    gf.close()
    gb.close()
    torch.cuda.synchronize()
    # every graph destroyed: the workspaces may be released and rebuilt
    _capi.check(_capi.lib().to_release())
    out = tp.propagate(fields[0], opts[0])
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(out)).all()
