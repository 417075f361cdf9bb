"""Host emulation of the large-block engine's GEMM staging indices
(bigeng.hpp: load_chunk / store_chunk and the matrix-core k-loop) for the
k-chunk widths 16, 32 and 64: every index stays inside the staging arrays
As / Bs [BG_KC][80] and the 64-row tile, and the 256 threads x BG_KC/4
registers cover the 64 x BG_KC chunk exactly once, for both operand
orientations.  (The 64-wide chunk is not built: it faulted the GPU once
with no cause found; this shows the index arithmetic is not that cause.)"""
import pytest

LDT = 64 + 16


@pytest.mark.parametrize("kc", [16, 32, 64])
@pytest.mark.parametrize("kfast", [True, False])
def test_staging_indices_in_bounds_and_bijective(kc, kfast):
    assert kc % 16 == 0 and 64 * kc == 256 * (kc // 4)
    seen = set()
    for t in range(256):
        for r in range(kc // 4):
            if kfast:
                kk, i = t % kc, t // kc + (256 // kc) * r
            else:
                i, kk = t & 63, (t >> 6) + 4 * r
            assert 0 <= kk < kc and 0 <= i < 64 and i < LDT
            seen.add((kk, i))
    assert len(seen) == 64 * kc


@pytest.mark.parametrize("kc", [16, 32, 64])
def test_matrix_core_loop_reads_inside_the_chunk(kc):
    for lane in range(64):
        for wv in range(4):
            wr, wc = wv >> 1, wv & 1
            for s in range(kc // 4):
                kr = 4 * s + (lane >> 4)
                assert 0 <= kr < kc
                for col in (wr * 32 + (lane & 15), wr * 32 + 16 + (lane & 15), wc * 32 + (lane & 15),
                            wc * 32 + 16 + (lane & 15)):
                    assert 0 <= col < 64 < LDT


def test_static_lds_of_the_wide_chunk_fits_the_device():
    """Static LDS of a large-block FP64 workgroup with a 64-wide chunk:
    two staged chunks, four 32 x 33 blocks of the factorization, two
    staging vectors, the reduction words and the function-scope arrays of
    the matrix-vector product and the sum (the compiler's resource report
    gives 121 936 bytes), below gfx950's 160 KiB per workgroup."""
    d = 8
    lds = (2 * 256 + 2 * 64 * LDT + 4 * 32 * 33) * d + 8 * 8 + 4 * 4 + 256 * d + 4 * d
    assert lds <= 121936 + 64 and lds < 160 * 1024
