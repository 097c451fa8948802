"""Host model of every LDS and red[] index of the single-workgroup path
(small_body in ntt.hip, run by k_small with one job per workgroup and by
k_small_persist with 2^(14-LG) jobs side by side in one 1024-thread workgroup).

The index formulas are restated here from the kernel source: SmallTile<LG>
(R = 2^LG values, NT = R/16 threads, 16 values per thread, LDS_WORDS = R + R/16
with one pad word per 16), the Stockham step radices and spans (radix-16 steps,
the leftover radix second in the forward transforms and last in the inverse),
the step loads (element j + t R/RAD of group j), the step stores (element
(j - j mod Ns) RAD + j mod Ns + t Ns), the final store of the inverse output,
lidx(r) = r + r/16, the group offsets g LDS_WORDS of the persistent kernel, and
red[2g], red[2g + 1]. For every LG and every group the test walks all indices
and checks them against the arrays the kernels declare: lds[LDS_WORDS] in
k_small, lds[2^14 + 2^10] and red[2 * 256] in k_small_persist.

It also records why a variant that ran the two forward transforms side by side,
each in its own tile of LDS_WORDS, cannot run in the persistent kernel as it is:
with the same group offsets its second tile overlaps the next group's tile, and
the last group's second tile lies past the array. The single-job kernel that
does run them side by side (k_small_pair, 2^10 to 2^13: the input's group in
the first tile of lds[2 LDS_WORDS], the seed's group in the second, the
input's spectrum handed over through the first tile, packing from the second)
is modelled the same way."""
import pytest

LDS_PERSIST = (1 << 14) + (1 << 10)
RED_PERSIST = 2 * 256


def radices(lg, inv):
    rf = (1 << (lg % 4)) if lg % 4 else 16
    nsteps = (lg + 3) // 4
    out = []
    for s in range(nsteps):
        if nsteps >= 3 and not inv:
            out.append(rf if s == 1 else 16)
        else:
            out.append((rf if s == nsteps - 1 else 16) if inv else (rf if s == 0 else 16))
    return out


def lidx(r):
    return r + (r >> 4)


def tile_indices(lg):
    """Every LDS index one job's small_body touches (relative to its tile)."""
    R = 1 << lg
    NT = R // 16
    idx = set()
    for inv in (False, True):
        rads = radices(lg, inv)
        ns = 1
        for s, rad in enumerate(rads):
            for lt in range(NT):
                for q in range(16 // rad):
                    j = lt + q * NT
                    if s > 0:  # loads of this step (written by the previous one)
                        idx.update(lidx(j + t * (R // rad)) for t in range(rad))
                    if s + 1 < len(rads):  # stores for the next step
                        jm = j & (ns - 1)
                        d = (j - jm) * rad + jm
                        idx.update(lidx(d + t * ns) for t in range(rad))
            ns *= rad
        if inv:  # the inverse output, stored for the parity and packing
            radi = rads[-1]
            for lt in range(NT):
                for q in range(16 // radi):
                    j = lt + q * NT
                    idx.update(lidx(j + t * (R // radi)) for t in range(radi))
    return idx


@pytest.mark.parametrize("lg", range(6, 15))
def test_every_index_stays_in_its_arrays(lg):
    R = 1 << lg
    words = R + R // 16
    idx = tile_indices(lg)
    assert min(idx) >= 0 and max(idx) < words          # k_small: lds[LDS_WORDS]
    assert len(idx) == R                               # every value has one slot
    jpw = 1 << (14 - lg)                               # jobs per persistent workgroup
    assert jpw * (R // 16) <= 1024                     # groups fit the 1024 threads
    top = max(g * words + i for g in range(jpw) for i in (max(idx),))
    assert top < LDS_PERSIST                           # k_small_persist: lds[2^14 + 2^10]
    assert 2 * (jpw - 1) + 1 < RED_PERSIST             # red[2 g], red[2 g + 1]
    # groups never share a word
    spans = [(g * words, g * words + max(idx)) for g in range(jpw)]
    assert all(a[1] < b[0] for a, b in zip(spans, spans[1:]))


@pytest.mark.parametrize("lg", range(6, 15))
def test_two_tiles_per_job_would_overrun_the_persistent_array(lg):
    R = 1 << lg
    words = R + R // 16
    jpw = 1 << (14 - lg)
    # second tile of group g at g * words + words, as the variant placed it
    second = [(g * words + words, g * words + 2 * words - 1) for g in range(jpw)]
    if jpw > 1:  # overlaps the next group's first tile
        assert second[0][0] == 1 * words
    assert second[-1][1] >= LDS_PERSIST  # the last group's second tile is past the array


@pytest.mark.parametrize("lg", range(10, 14))
def test_pair_kernel_indices_stay_in_their_tiles(lg):
    R = 1 << lg
    NT = R // 16
    words = R + R // 16
    assert NT >= 64 and 2 * NT <= 1024                  # groups of whole waves in one workgroup
    per_tile = tile_indices(lg)                         # both groups' steps (a superset for the input's)
    radl = radices(lg, False)[-1]
    handover = set()                                    # the input's spectrum, written and read in tile 0
    for lt in range(NT):
        for q in range(16 // radl):
            j = lt + q * NT
            handover.update(lidx(j + t * (R // radl)) for t in range(radl))
    assert len(handover) == R and handover <= per_tile
    packing = {lidx(i) for i in range(R)}               # out[lidx(i)], i < m <= R, in tile 1
    assert packing <= per_tile
    for g in (0, 1):
        absolute = {g * words + i for i in per_tile | (handover if g == 0 else packing)}
        assert min(absolute) >= g * words and max(absolute) < (g + 1) * words
    assert 2 * words * 4 <= 160 * 1024                  # lds[2 LDS_WORDS] fits one CU
