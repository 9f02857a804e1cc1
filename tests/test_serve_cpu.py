"""Host logic of the server (CPU only): the arena allocator that carves the
HBM budget, checked against a brute-force model of the byte range."""
import numpy as np

from paper_0912_2555_amd import serve


def test_arena_first_fit_and_coalescing():
    a = serve.Arena(4096)
    x = a.alloc(1000)            # rounded to 1024
    y = a.alloc(256)
    z = a.alloc(2000)            # 2048
    assert (x, y, z) == (0, 1024, 1280)
    assert a.alloc(1024) is None  # 768 bytes left
    a.free(y, 256)
    assert a.alloc(800) is None   # holes of 256 (at 1024) and 768 (at 3328), not adjacent
    assert a.alloc(200) == 1024   # first fit takes the lower hole
    a.free(1024, 200)
    a.free(x, 1000)               # merges with the 256 hole
    assert a.alloc(1280) == 0
    a.free(0, 1280)
    a.free(z, 2000)
    assert a.free_off == [0] and a.free_len == {0: 4096}


def test_arena_random_against_model():
    rng = np.random.default_rng(5)
    size = 1 << 16
    a = serve.Arena(size)
    used = np.zeros(size // 256, bool)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off, nb = live.pop(int(rng.integers(len(live))))
            a.free(off, nb)
            used[off // 256:(off + nb) // 256] = False
        else:
            nb = int(rng.integers(1, 8)) * 256
            off = a.alloc(nb)
            # first fit: the lowest run of free 256-byte units that is long enough
            k = nb // 256
            runs = [i for i in range(len(used) - k + 1) if not used[i:i + k].any()]
            if off is None:
                assert not runs
                continue
            assert off == runs[0] * 256
            assert not used[off // 256:(off + nb) // 256].any()
            used[off // 256:(off + nb) // 256] = True
            live.append((off, nb))
        assert a.free_bytes() == (~used).sum() * 256
        # free ranges are maximal: no two touch
        for o1, o2 in zip(a.free_off, a.free_off[1:]):
            assert o1 + a.free_len[o1] < o2


def test_footprint_covers_every_buffer():
    lay, total = serve._layout(1000, 5000)
    assert set(lay) == {"row_ptr", "col", "scratch"}          # edges and flags stay in pinned host memory
    ends = sorted((o, o + ln) for o, ln in lay.values())
    for (o1, e1), (o2, _) in zip(ends, ends[1:]):
        assert e1 <= o2 and o2 % 256 == 0
    assert ends[-1][1] <= total == serve.footprint(1000, 5000)
