"""Position maps of the register passes (Section III, the Kronecker structure
of eq. (6) that makes each group of stages block-diagonal), checked by brute
force on the CPU: which threads an LDS exchange between two passes connects.

The kernels order an exchange with wave-level synchronisation only (no
workgroup barrier) when it cannot leave a wave: between two full passes the
exchange into the pass after stage S stays inside aligned runs of 2^S
consecutive threads, so with 2^S <= 64 every run is inside one 64-lane wave.
In the decimation-in-frequency order (eq. (9)) the passes run from the top
bits down, and the exchange into the pass on bits S .. S+RB-1 stays inside
aligned runs of 2^(S+RB) threads: there the last exchanges are the local ones.
These tests enumerate every position and confirm both rules, and that they are
sharp (every other exchange does cross waves)."""
import pytest


def position(lt, s, rp, t, u):
    g, uu = u >> rp, u & ((1 << rp) - 1)
    o = t + (g << lt)
    return (o & ((1 << s) - 1)) + (uu << s) + ((o >> s) << (s + rp))


def passes(m, rb):
    out, s = [], 0
    while s < m:
        rp = rb if s + rb <= m else m - s
        out.append((s, rp))
        s += rp
    return out


def holder(m, rb, p):
    """Position -> thread of pass p."""
    lt = m - rb
    s, rp = passes(m, rb)[p]
    where = {}
    for t in range(1 << lt):
        for u in range(1 << rb):
            j = position(lt, s, rp, t, u)
            assert j not in where
            where[j] = t
    assert len(where) == 1 << m
    return where


def wave_local(m, rb, p):
    """The kernels' rule (a group whose threads are the consecutive lanes of
    aligned runs): pass p full, 2^S <= 64, more than one wave of threads."""
    ps = passes(m, rb)
    if not 1 <= p < len(ps):
        return False
    s, rp = ps[p]
    return (1 << (m - rb)) > 64 and rp == rb and (1 << s) <= 64


CASES = [(m, rb) for rb in (3, 4, 5) for m in range(rb + 1, 17) if (1 << (m - rb)) <= 4096]


@pytest.mark.parametrize("m,rb", CASES)
def test_exchange_stays_in_aligned_runs(m, rb):
    ps = passes(m, rb)
    for p in range(1, len(ps)):
        s, rp = ps[p]
        if rp != rb:
            continue
        a, b = holder(m, rb, p - 1), holder(m, rb, p)
        for j in range(1 << m):
            assert a[j] >> s == b[j] >> s, (m, rb, p, j)


@pytest.mark.parametrize("m,rb", CASES)
def test_wave_local_rule_is_exact(m, rb):
    ps = passes(m, rb)
    for p in range(1, len(ps)):
        a, b = holder(m, rb, p - 1), holder(m, rb, p)
        crosses = any(a[j] >> 6 != b[j] >> 6 for j in range(1 << m))
        if wave_local(m, rb, p):
            assert not crosses, (m, rb, p)
        elif (1 << (m - rb)) > 64 and ps[p][1] == rb:
            # full passes with 2^S > 64: the exchange does reach other waves
            assert crosses, (m, rb, p)


def test_rule_covers_the_first_exchange_of_the_long_single_pass_lengths():
    # 16 elements per thread: 2^11 .. 2^14 have more than one wave of threads
    # per transform, and their first exchange (after stage 4) is wave-local
    for m in (11, 12, 13, 14):
        assert wave_local(m, 4, 1)
        assert not wave_local(m, 4, 2)
    # 32 elements per thread: after stage 5, runs of 32 threads
    for m in (12, 13, 14, 15):
        assert wave_local(m, 5, 1)


def passes_dif(m, rb):
    np_ = (m + rb - 1) // rb
    rp0 = m - rb * (np_ - 1)
    return [(m - rp0 - rb * p, rp0 if p == 0 else rb) for p in range(np_)]


def holder_dif(m, rb, p):
    lt = m - rb
    s, rp = passes_dif(m, rb)[p]
    where = {}
    for t in range(1 << lt):
        for u in range(1 << rb):
            j = position(lt, s, rp, t, u)
            assert j not in where
            where[j] = t
    assert len(where) == 1 << m
    return where


def dif_wave_local(m, rb, p):
    """The kernels' DIF rule: pass p-1 full, 2^(S+RB) <= 64 for pass p's S,
    more than one wave of threads."""
    ps = passes_dif(m, rb)
    if not 1 <= p < len(ps):
        return False
    return (1 << (m - rb)) > 64 and ps[p - 1][1] == rb and (1 << (ps[p][0] + rb)) <= 64


@pytest.mark.parametrize("m,rb", CASES)
def test_dif_exchange_stays_in_aligned_runs(m, rb):
    ps = passes_dif(m, rb)
    for p in range(1, len(ps)):
        s = ps[p][0]
        if ps[p - 1][1] != rb:
            continue
        a, b = holder_dif(m, rb, p - 1), holder_dif(m, rb, p)
        for j in range(1 << m):
            assert a[j] >> (s + rb) == b[j] >> (s + rb), (m, rb, p, j)


@pytest.mark.parametrize("m,rb", CASES)
def test_dif_wave_local_rule_is_exact(m, rb):
    ps = passes_dif(m, rb)
    for p in range(1, len(ps)):
        a, b = holder_dif(m, rb, p - 1), holder_dif(m, rb, p)
        crosses = any(a[j] >> 6 != b[j] >> 6 for j in range(1 << m))
        if dif_wave_local(m, rb, p):
            assert not crosses, (m, rb, p)
        elif (1 << (m - rb)) > 64:
            assert crosses, (m, rb, p)


def test_dif_rule_covers_the_last_exchange():
    for m in (11, 12, 13, 14):
        last = len(passes_dif(m, 4)) - 1
        assert dif_wave_local(m, 4, last)
        assert not any(dif_wave_local(m, 4, p) for p in range(1, last))
    for m in (12, 13, 14):
        assert dif_wave_local(m, 5, len(passes_dif(m, 5)) - 1)
