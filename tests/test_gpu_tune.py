"""The strategy search (rise_autotune_gemm / rise_autotune_stencil) and its
cache: the tuner records one of the supported tiles / schedules for the key
(sizes, mode, architecture); once the cache is set, the calls that leave the
choice to the library run that entry -- the host query reports it, the default
call gives the same bits as the call with the entry passed explicitly, and both
meet the oracle's parity bar."""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, gemm_scale, host, stencil_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    yield rise
    rise.rise_set_tune_cache(None)


def cache_lines(path, kind):
    return [l.split() for l in open(path).read().splitlines() if l.startswith(kind + " ")]


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_autotune_gemm_entry_is_what_runs(rise, tmp_path, mode):
    M, N, K = 1000, 1200, 700
    path = str(tmp_path / "tune.txt")
    print(f"autotune gemm {M}x{N}x{K} mode={mode}", flush=True)
    rise.rise_autotune_gemm(path, M, N, K, mode)
    rise.rise_autotune_gemm(path, 256, 256, 256, mode)  # a second key is kept beside it
    lines = cache_lines(path, "gemm")
    assert len(lines) == 2 and {l[1] for l in lines} == {"gfx950"}
    e = [l for l in lines if l[2:5] == [str(M), str(N), str(K)]][0]
    tile = tuple(int(v) for v in e[6:9])
    assert tile in rise.rise_gemm_tiles(mode)
    rise.rise_set_tune_cache(path)
    assert rise.rise_gemm_default_tile(M, N, K, mode) == tile
    assert rise.rise_gemm_workspace(M, N, K, mode) == rise.rise_gemm_workspace(M, N, K, mode, tile)
    A, B = ri.gemm_uniform(M, N, K, 4300 + K)
    want = host(rise.gemm(dev(A), dev(B), mode=mode))
    got = host(rise.gemm(dev(A), dev(B), mode=mode, tile=tile))
    rise.rise_set_tune_cache(None)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert componentwise(want, oracle.gemm(A, B), gemm_scale(A, B)) <= 1e-5


def test_gemm_cache_entry_overrides_the_default(rise, tmp_path):
    # a hand-written entry for a tile other than the built-in default is reported
    # and run (the workspace query follows it: bf16x3 pads to whole tiles)
    M, N, K = 1000, 1200, 700
    default = rise.rise_gemm_default_tile(M, N, K, "bf16x3")
    other = [t for t in rise.rise_gemm_tiles("bf16x3") if t != default][0]
    path = tmp_path / "tune.txt"
    path.write_text(f"gemm gfx950 {M} {N} {K} 2 {other[0]} {other[1]} {other[2]} 1.0\n")
    rise.rise_set_tune_cache(str(path))
    try:
        assert rise.rise_gemm_default_tile(M, N, K, "bf16x3") == other
        assert rise.rise_gemm_workspace(M, N, K, "bf16x3") == \
            rise.rise_gemm_workspace(M, N, K, "bf16x3", other)
        A, B = ri.gemm_uniform(M, N, K, 4400)
        got = host(rise.gemm(dev(A), dev(B), mode="bf16x3"))
        assert componentwise(got, oracle.gemm(A, B), gemm_scale(A, B)) <= 1e-5
        # another architecture's entry is not used
        path.write_text(f"gemm gfx942 {M} {N} {K} 2 {other[0]} {other[1]} {other[2]} 1.0\n")
        rise.rise_set_tune_cache(str(path))
        assert rise.rise_gemm_default_tile(M, N, K, "bf16x3") == default
    finally:
        rise.rise_set_tune_cache(None)


@pytest.mark.parametrize("k", [3, 5])
def test_autotune_stencil_entry_is_what_runs(rise, tmp_path, k):
    H, W = 700, 900
    path = str(tmp_path / "tune.txt")
    print(f"autotune stencil {H}x{W} k={k}", flush=True)
    rise.rise_autotune_stencil(path, H, W, k)
    lines = cache_lines(path, "stencil")
    assert len(lines) == 1 and lines[0][1] == "gfx950"
    names = {v: n for n, v in rise.SCHEDULES.items()}
    sched = (names[int(lines[0][5])], int(lines[0][6]))
    assert sched in rise.rise_stencil_schedules()
    rise.rise_set_tune_cache(path)
    assert rise.rise_stencil2d_default_schedule(H, W, k, k) == sched
    img = ri.uniform_matrix(ri.rng(H + k), H, W, 0.0, 1.0)
    w = ri.random_weights(ri.rng(k), k)
    want = host(rise.stencil2d(dev(img), dev(w)))
    got = host(rise.stencil2d(dev(img), dev(w), schedule=sched))
    rise.rise_set_tune_cache(None)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert componentwise(want, oracle.stencil2d(img, w), stencil_scale(img, w, oracle.PAD_CLAMP)) <= 1e-5
