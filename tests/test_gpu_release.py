"""to_release frees every workspace and table of the library (scratch,
partials, transfer tables, DI and Bluestein tables, resampling tables,
private accumulators) and the next calls rebuild them: results after a
release equal those before, bitwise."""
import numpy as np
import pytest

from tests._util import announce, crandn, to_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_release_and_rebuild():
    import paper_2411_18591_amd as tp
    announce("release and rebuild")
    rng = np.random.default_rng(1300)
    u = to_gpu(crandn(rng, 3, 40, 48, dtype=np.complex64), torch)
    asm = tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=2e-3, pad=2)
    di = tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=0.02, method="di", pad=2)
    odd = tp.Optics(dy=4e-6, dx=4e-6, wavelength=0.6e-6, z=2e-3, pad=2, round_pow2=False)
    I = torch.zeros((3, 40, 48), dtype=torch.float32, device="cuda")

    def run():
        outs = tp.propagate_jobs([u, u, u], [asm, di, odd])
        I.zero_()
        jobs = [tp.make_job(u, o, epi=tp._capi.TO_EPI_INTENSITY, epi_out=I, epi_scale=1.0)
                for o in (asm, di, asm)]
        tp._capi.propagate(jobs, tp._capi.TO_C64, torch.cuda.current_stream().cuda_stream)
        r = tp.resample(outs[0], tp.Grid(40, 48, 4e-6, 4e-6), tp.Grid(50, 30, 3e-6, 5e-6))
        torch.cuda.synchronize()
        return [o.clone() for o in outs] + [I.clone(), r]

    before = run()
    tp._capi.check(tp._capi.lib().to_release())
    after = run()
    for a, b in zip(before, after):
        assert torch.equal(a, b)
