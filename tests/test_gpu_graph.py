"""Graph capture of the single-mesh path.  A step followed by the TV
indicator (with the single-workgroup statistics on a small mesh and the
multi-workgroup ones above 65,536 cells), and the allocation-free step, are
captured once with torch.cuda.graph and replayed several times, with eager
work and synchronisations between the replays; every replay gives the bits
of the same calls made eagerly."""
import pytest

torch = pytest.importorskip("torch")

from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I

pytestmark = pytest.mark.gpu


def _mesh(w):
    m = adg.Mesh(w["phys"], w["mesh"])
    m.init_state("bubbles", w["bubbles"])
    m.compute_dt()
    return m


def _tv_buffers(C):
    return (torch.zeros(C, dtype=torch.float64, device="cuda"), torch.zeros(C, dtype=torch.int8, device="cuda"),
            torch.zeros(3, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("nx,N", [(9, 6), (27, 6), (260, 2)])
def test_step_and_tv_indicator_graph_replays_equal_eager(nx, N):
    """9x9 and 27x27 at N = 6 (the one-wavefront-per-level and the
    four-wavefronts-per-cell predictors), 260x260 at N = 2 (67,600 cells:
    one wavefront per cell, statistics through per-workgroup partials)."""
    w = I.bubble(nx, N, bubbles=[I.cosine_bubble(), I.cold_bubble()])
    eager, cap = _mesh(w), _mesh(w)
    C = eager.C
    te, tg = _tv_buffers(C), _tv_buffers(C)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cap.step(s)
        cap.tv_indicator(adg.ADG_VAR_THETA, 1.0, 0.0, *tg, s)
    torch.cuda.synchronize()
    for k in range(4):
        eager.step()
        eager.tv_indicator(adg.ADG_VAR_THETA, 1.0, 0.0, *te)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eager.Q, cap.Q), k
        assert torch.equal(eager.clock, cap.clock), k
        for a, b in zip(te, tg):
            assert torch.equal(a, b), k
        assert tg[2][0].item() == C and (tg[1] == 1).any()


def test_static_step_graph_replays_equal_eager():
    """The allocation-free step captured and replayed against adg_step_static
    called eagerly on a second copy of the state."""
    w = I.bubble(27, 6)
    m = _mesh(w)
    Qe, ce = m.Q.clone(), m.clock.clone()
    Qg, cg = m.Q.clone(), m.clock.clone()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.step_static(Qg, cg, s)
    torch.cuda.synchronize()
    for k in range(4):
        m.step_static(Qe, ce)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Qe, Qg), k
        assert torch.equal(ce, cg), k
        assert cg[3].item() == k + 1
