"""Host-side checks of the chunk partition (Section 3.1.1, Algorithm 3) that the
kernels rely on: with power-of-two chunks every thread flips the same column
at every local step (the paper's CEG claim), and with the kernels' lane
numbering the flip's sign is the same across the 64 lanes of a wave too, so
a column and its sign are wave-uniform (scalar loads, no divergence).  Pure
host logic: no GPU, no oracle arithmetic."""


def ctz(g: int) -> int:
    return (g & -g).bit_length() - 1


def gray(g: int) -> int:
    return g ^ (g >> 1)


def distinct_columns(chunk: int, threads: int):
    # thread t walks g = t * chunk + 1 + i, i = 0 .. chunk - 1 (Algorithm 3's
    # start without the remainder), and flips column ctz(g) at local step i
    return [len({ctz(t * chunk + 1 + i) for t in range(threads)}) for i in range(chunk)]


def test_paper_ceg_claims():
    # Section 3.1.1: a chunk of 17 over 4 threads gives 3 different columns at
    # every local iteration; a chunk of 16 gives one column except the last
    assert distinct_columns(17, 4) == [3] * 17
    assert distinct_columns(16, 4) == [1] * 15 + [3]


def lane_chunk_index(wave: int, lane: int) -> int:
    # the kernels' numbering: bit 0 of the chunk index is the wave's parity,
    # bits 1..6 the lane, the rest the wave pair
    return (wave & 1) | (lane << 1) | ((wave >> 1) << 7)


def test_flip_and_sign_are_wave_uniform():
    for c in (4, 5, 7, 9):
        for wave in range(6):
            for l in range(1, 1 << c):
                cols, signs = set(), set()
                for lane in range(64):
                    g = (lane_chunk_index(wave, lane) << c) | l
                    j = ctz(g)
                    cols.add(j)
                    signs.add((gray(g) >> j) & 1)  # 1: the column enters S
                assert cols == {ctz(l)}, (c, wave, l)
                assert len(signs) == 1, (c, wave, l)


def test_lanes_tile_the_walk_exactly():
    # lanes x 2^c = 2^(n-1): every Gray index is visited once, no remainder
    n, c = 14, 5
    waves = (1 << (n - 1 - c)) // 64
    seen = set()
    for wave in range(waves):
        for lane in range(64):
            k = lane_chunk_index(wave, lane)
            seen.update(range(k << c, (k + 1) << c))
    assert seen == set(range(1 << (n - 1)))
