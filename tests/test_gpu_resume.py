"""Checkpoint / resume of the decoder state (mpd_run_steps_from): a state
exported after t1 steps and resumed for t2 more equals a straight run of
t1 + t2 steps (and the oracle's), for the plain rule and the limited-memory
variant, in place or not, in one resume or several."""
import numpy as np
import pytest
import torch

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


def patterns(orc, L, p, n, tag):
    ms = seeds(180, 1000 * tag + L, n)
    exs, eys = zip(*[orc.noise(L, p, int(x)) for x in ms])
    return ms, exs, eys, orc.links_from_chains(L, np.stack(exs), np.stack(eys))


@pytest.mark.parametrize("L,p,n", [(3, 0.2, 16), (8, 0.08, 32), (16, 0.06, 16), (30, 0.05, 8), (64, 0.04, 8),
                                   (128, 0.03, 4)])
def test_resume_equals_a_straight_run(gpu, orc, L, p, n):
    ms, exs, eys, links = patterns(orc, L, p, n, 1)
    for t1, t2 in ((0, 5), (3, 4), (7, 0), (2, 9)):
        M1, S1, W1 = gpu.run_steps(L, links, t1)
        M2, S2, W2 = gpu.run_steps_from(L, M1, S1, W1, t1, t2)
        Mr, Sr, Wr = gpu.run_steps(L, links, t1 + t2)
        assert torch.equal(M2, Mr) and torch.equal(S2, Sr) and torch.equal(W2, Wr), (L, t1, t2)
    m, sig, _, _ = orc.run_steps(L, exs[0], eys[0], 11)
    assert np.array_equal(M2[0].cpu().numpy().astype(np.int64), m.astype(np.int64))


def test_resume_in_place_and_in_chunks(gpu, orc):
    L = 32
    _, _, _, links = patterns(orc, L, 0.07, 24, 2)
    M, S, W = gpu.run_steps(L, links, 2)
    t = 2
    for k in (1, 3, 2, 5):
        gpu.run_steps_from(L, M, S, W, t, k, out=(M, S, W))
        t += k
    Mr, Sr, Wr = gpu.run_steps(L, links, t)
    assert torch.equal(M, Mr) and torch.equal(S, Sr) and torch.equal(W, Wr)


@pytest.mark.parametrize("m_max,u", [(3, 0), (0, 2), (4, 3)])
@pytest.mark.parametrize("L", [9, 64])
def test_resume_keeps_the_step_numbers_of_the_rule_variant(gpu, orc, L, m_max, u):
    """Truncation and random moves depend on the absolute step: resuming at
    t1 gives the straight run's state, and the oracle's."""
    ms, exs, eys, links = patterns(orc, L, 0.07, 6, 3)
    for t1, t2 in ((1, 5), (4, 4)):
        M1, S1, W1 = gpu.run_steps(L, links, t1, m_max=m_max, u=u, move_seeds=ms)
        M2, S2, W2 = gpu.run_steps_from(L, M1, S1, W1, t1, t2, m_max=m_max, u=u, move_seeds=ms)
        Mr, Sr, Wr = gpu.run_steps(L, links, t1 + t2, m_max=m_max, u=u, move_seeds=ms)
        assert torch.equal(M2, Mr) and torch.equal(S2, Sr) and torch.equal(W2, Wr), (t1, t2)
        m, sig, _, _ = orc.run_steps(L, exs[1], eys[1], t1 + t2, m_max=m_max, u=u, seed=int(ms[1]))
        assert np.array_equal(M2[1].cpu().numpy().astype(np.int64), m.astype(np.int64))


@pytest.mark.parametrize("L", [64, 80, 96])
def test_strip_table_sizes_in_every_mode(gpu, orc, L):
    """The lattice sizes whose strip height is set by the measured table
    (64 -> 8, 80 -> 10, 96 -> 12): seeded decodes of the plain rule, the
    limited-memory rule and the open lattice, and a state export, against
    the oracle."""
    n = 6
    s = seeds(181, L, n)
    for kw, okw, fn in ((dict(), dict(), gpu.decode_batch),
                        (dict(m_max=4, u=3), dict(m_max=4, u=3), gpu.decode_rule),
                        (dict(), dict(open_bc=True), gpu.decode_open)):
        T, F, S = fn(L, 0.05, s, 300, **kw)
        ref = orc.decode_seeds(L, 0.05, s, 300, threads=8, **okw)
        assert np.array_equal(T.cpu().numpy(), ref["T_dec"]) and np.array_equal(F.cpu().numpy(), ref["flags"]), fn
        assert np.array_equal(S.cpu().numpy().view(np.uint32), ref["sigma_words"]), fn
    ms, exs, eys, links = patterns(orc, L, 0.06, 2, 4)
    M, S, W = gpu.run_steps(L, links, 5)
    m, sig, _, _ = orc.run_steps(L, exs[0], eys[0], 5)
    assert np.array_equal(M[0].cpu().numpy().astype(np.int64), m.astype(np.int64))
