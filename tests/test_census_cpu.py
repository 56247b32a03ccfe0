"""CPU checks of the census helper that GPU tests compare the pair kernel's
neighbour census with: the id mixing function against published SplitMix64
outputs, the expected sets against the O(N^2) brute force and the oracle's
bucket search, and the subset matching of ambiguous pairs."""
import numpy as np

import sph_synth as S
from oracle import cpu
from tests import brute
from tests.census import expected, match, mix64, sum64


def test_mix64_is_splitmix64():
    # SplitMix64 seeded with 0 yields these first two outputs; mix64(k) is the
    # output function applied to k + the golden-ratio increment
    assert int(mix64([0])[0]) == 0xE220A8397B1DCDAF
    assert int(mix64([0x9E3779B97F4A7C15])[0]) == 0x6E789E6AA1B965F4
    # a bijection: distinct ids give distinct words on a sample
    v = mix64(np.arange(100000))
    assert np.unique(v).size == v.size


def test_expected_sets_equal_brute_force_and_oracle():
    wl = S.random_cloud(700, seed=71, h=0.05)
    st = cpu.State.from_workload(wl)
    o, _, start = cpu.build_cells(wl.grid, st)
    ex = expected(o.x, o.x, wl.params["h"])
    got = {(i, int(j)) for i, js in enumerate(ex.core) for j in js if j != i}
    assert got == brute.neighbor_pairs(o.x, o.x, wl.params["h"], True)
    pi, pj = cpu.neighbors(wl.params, wl.grid, o, o, start, True)
    assert got == set(zip(pi.tolist(), pj.tolist()))
    # every target lists itself (r = 0 is evaluated and adds nothing)
    assert all(i in set(js.tolist()) for i, js in enumerate(ex.core))


def test_match_finds_the_ambiguous_subset():
    core = np.array([3, 7, 11])
    amb = np.array([20, 21])
    amb_in = np.array([True, False])
    ids = np.arange(40)
    s_core = sum64(mix64(ids[core]))
    # the device agrees with FP64 on both ambiguous pairs
    assert match(4, (s_core + int(mix64([20])[0])) & (2**64 - 1), ids[core], ids[amb], amb_in) == 0
    # the device takes the outer one instead of the inner one
    assert match(4, (s_core + int(mix64([21])[0])) & (2**64 - 1), ids[core], ids[amb], amb_in) == 2
    # a lost core neighbour is not explained by any subset
    assert match(2, sum64(mix64(ids[core[:2]])), ids[core], ids[amb], amb_in) is None
