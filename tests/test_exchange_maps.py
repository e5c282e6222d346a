"""Position maps of the register passes (Section III, the Kronecker structure
of eq. (6) that makes each group of stages block-diagonal), checked by brute
force on the CPU: which threads an LDS exchange between two passes connects.

The kernels order an exchange with wave-level synchronisation only (no
workgroup barrier) when it cannot leave a wave: between two full passes the
exchange into the pass after stage S stays inside aligned runs of 2^S
consecutive threads, so with 2^S <= 64 every run is inside one 64-lane wave.
These tests enumerate every position and confirm that rule, and that it is
sharp (the next exchange does cross waves)."""
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
