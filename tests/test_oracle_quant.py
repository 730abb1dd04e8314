"""Pin the reduced-storage emulation: RNE conversions against library
routines (numpy float16, torch bfloat16), the scale rule, and the block
structure of the emulation."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import workload as W


def _probe_values(rng):
    v = [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.99, 65520.0, -65520.0, 6.1e-5, 5.96e-8, 2.98e-8,
         2.9802322e-08, 1e-30, 3.0e38, 1.5, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14]
    # exact fp16 ties: midpoints between adjacent fp16 values, all exponents
    h = np.arange(0, 0x7bff, 37, dtype=np.uint16).view(np.float16).astype(np.float32)
    h2 = (np.arange(1, 0x7c00, 37, dtype=np.uint16)).view(np.float16).astype(np.float32)
    n = min(len(h), len(h2))
    mids = (h[:n].astype(np.float64) + h2[:n].astype(np.float64)) / 2
    v += list(mids.astype(np.float32))
    v += list((rng.standard_normal(20000) * np.exp(rng.uniform(-40, 14, 20000))).astype(np.float32))
    x = np.array(v, dtype=np.float32)
    return np.concatenate([x, -x])


def test_fp16_rne_matches_numpy():
    rng = np.random.default_rng(0)
    x = _probe_values(rng)
    ours = oracle.quantize_bits(1, x)
    ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_rne_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = _probe_values(rng)
    x = np.concatenate([x, (rng.standard_normal(20000) * 1e30).astype(np.float32)])
    ours = oracle.quantize_bits(2, x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("m,a,s", [((1.0,) * 6, 0.0, 10), ((1.5,) * 6, 0.0, 9), ((2.0,) * 6, 0.0, 9),
                                   ((0.75,) * 6, 0.0, 10), ((0.0,) * 6, 0.0, 0), ((0.0,) * 6, 0.75, 10),
                                   ((0.0,) * 6, 3.0, 8), ((1e-30,) * 6, 0.0, 64), ((1e30,) * 6, 0.0, -64),
                                   ((65504.0,) * 6, 0.0, -6), ((0.5,) * 6, 4.0, 8)])
def test_scale_rule(m, a, s):
    assert list(oracle.choose_scales(m, a)) == [s] * 6


def test_scale_rule_zero_component_takes_largest():
    """A zero component with no sources takes the largest component maximum."""
    s = oracle.choose_scales([0.0, 3.0, 0.5, 0.0, 0.0, 0.0], 0.0)
    assert list(s) == [8, 8, 11, 8, 8, 8]


def _small_problem():
    wl = W.spheres(10, 9, 8, 3, 24, seed=77, n_sources=1, n_probes=4, rmin=1, rmax=3)
    return wl, oracle.Problem.from_workload(wl)


@pytest.mark.parametrize("fmt", [1, 2])
def test_one_block_equals_f32_then_quantize(fmt):
    wl, prob = _small_problem()
    f = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    st = prob.quantize_upload(f, fmt)
    g = f.copy()
    pq = prob.run_q(f, 0, 24, fmt, 1000, st)
    p32 = prob.run_f32(g, 0, 24)
    assert np.array_equal(pq, p32)          # probes see the f32 working values
    st2 = {"scales": np.zeros(6, np.int32), "m_stored": np.zeros(6, np.float32), "flag": np.zeros(1, np.int32)}
    st2["m_stored"][:] = 0.0
    oracle.lib().orc_quantize_state(wl.nx, wl.ny, wl.nz, fmt, 0, prob.a_max, g,
                                    st2["scales"], st2["m_stored"], st2["flag"])
    assert np.array_equal(f, g)
    # stored values are exactly representable after scaling
    for c in range(6):
        y = f[c] * np.float32(2.0 ** int(st["scales"][c]))
        if fmt == 1:
            assert np.array_equal(y.astype(np.float16).astype(np.float32), y)
        else:
            assert np.all((y.view(np.uint32) & 0xFFFF) == 0)


def test_block_boundaries_change_result_and_t_matters():
    wl, prob = _small_problem()
    outs = []
    for T in (1, 4):
        f = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
        st = prob.quantize_upload(f, 1)
        prob.run_q(f, 0, 24, 1, T, st)
        outs.append(f)
    f32 = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    prob.run_f32(f32, 0, 24)
    assert not np.array_equal(outs[0], outs[1])
    e1, e4 = W.rel_l2(outs[0], f32), W.rel_l2(outs[1], f32)
    assert 0 < e4 < e1 < 1e-2


def test_overflow_block_retried_with_its_own_scale():
    """A component whose stored maximum is tiny, driven hard by H within one
    block, would exceed the 64x headroom at the block's end: that component
    is quantised instead with the scale of its own end-of-block maximum,
    10 - ceil(log2 max(m', A)), and nothing saturates (the overflow retry).
    Checked against the same block in plain FP32 quantised by numpy's
    binary16 (RNE), with the scale computed here from frexp; the other
    components keep the scale rule's choice.  bfloat16 has the range of
    binary32 and keeps the rule's scales."""
    wl, _ = _small_problem()
    p = oracle.Problem(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, wl.eps_r, wl.sigma, wl.mat)
    for fmt in (1, 2):
        f = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
        f[3, 3:5, 3:5, 3:6] = 1.0               # Hx block
        f[2, 2, 2, 2] = 1e-6                    # Ez max 1e-6 -> scale 10+19 = 29
        st = p.quantize_upload(f, fmt)
        assert st["scales"][2] == 29
        rule = oracle.choose_scales(st["m_stored"], 0.0)     # the scales the rule picks for this block
        g = f.copy()
        p.run_q(f, 0, 2, fmt, 2, st)
        p.run_f32(g, 0, 2)                      # the block's own values, before quantisation
        assert st["flag"][0] == 0
        for c in range(6):
            x = g[c].astype(np.float64)
            if fmt == 1 and np.max(np.abs(x)) * 2.0 ** rule[c] >= 65520.0:
                fr, e = np.frexp(np.max(np.abs(x)))
                sc = 10 - (e - 1 if fr == 0.5 else e)
                assert c == 2 and sc < 29 - 6       # Ez grew far past its headroom
            else:
                sc = rule[c]
            assert st["scales"][c] == sc, c
            if fmt == 1:
                q = (g[c] * np.float32(2.0 ** sc)).astype(np.float16).astype(np.float32) * np.float32(2.0 ** -sc)
                assert np.array_equal(f[c], q), c
        if fmt == 1:
            assert np.max(np.abs(f[2])) < 1024.0 * 2.0 ** -st["scales"][2]


def test_non_finite_value_still_flags():
    """A NaN cannot be stored: the flag is raised whatever the retry."""
    wl, _ = _small_problem()
    p = oracle.Problem(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, wl.eps_r, wl.sigma, wl.mat)
    f = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    f[3, 3:5, 3:5, 3:6] = 1.0
    st = p.quantize_upload(f, 1)
    f[4, 4, 4, 4] = np.nan
    p.run_q(f, 0, 2, 1, 2, st)
    assert st["flag"][0] == 1