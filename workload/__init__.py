"""Seeded synthetic inputs for the virtual-PE SHMEM workloads.

This module is the only code shared by the CPU oracle and the GPU path.  It
draws random numbers and lays out operation lists; it performs none of the
SHMEM operations themselves (no copies between PEs, no atomics, no
reductions).

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), in its counter form:
output ``i`` (0-based) of the stream seeded with ``s`` is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` where ``mix`` is the 64-bit
finaliser of that paper.  Because the stream is counter-based, any window of
it can be produced without producing its prefix.

Bounded integers use Lemire's multiply-shift (Lemire, "Fast random integer
generation in an interval", ACM TOMACS 2019, without the rejection step):
``a + ((x * (b - a + 1)) >> 64)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Base seeds of the five workloads.
SEED_SMALL = 0x5EED0001      # 4 PEs x 1 MiB, mixed put/get + contended fetch_add
SEED_SWEEP = 0x5EED0002      # 64 PEs x 1 GiB bandwidth sweep
SEED_GUPS = 0x5EED0003       # random-access AMOs + ping-pong
SEED_COLL = 0x5EED0004       # team collectives over 64 PEs
SEED_SERVE = 0x5EED0005      # serving / batching mix

# Sub-stream tags: subseed(base, tag).
TAG_OPS = 1
TAG_AMO = 2
TAG_PERM = 3
TAG_SIZES = 4
TAG_ARRIVAL = 5
TAG_HEAP = 0x100            # + pe


# ---------------------------------------------------------------- SplitMix64
def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _MASK64) + idx * GOLDEN
    return _mix(state)


def splitmix64_scalar(seed: int, i: int) -> int:
    """Output ``i`` of the stream of ``seed`` as a Python int (pure integer code)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def subseed(base: int, tag: int) -> int:
    """Seed of the sub-stream ``tag`` of workload ``base``: output 0 of base^tag."""
    return splitmix64_scalar((base ^ tag) & _MASK64, 0)


def mulhi64(x: np.ndarray, m: int) -> np.ndarray:
    """High 64 bits of the 128-bit product x*m (x uint64 array, 0 <= m < 2^64)."""
    x = np.asarray(x, dtype=np.uint64)
    m = int(m)
    lo32 = np.uint64(0xFFFFFFFF)
    x0 = x & lo32
    x1 = x >> np.uint64(32)
    m0 = np.uint64(m & 0xFFFFFFFF)
    m1 = np.uint64(m >> 32)
    with np.errstate(over="ignore"):
        p00 = x0 * m0
        p01 = x0 * m1
        p10 = x1 * m0
        p11 = x1 * m1
        mid = (p00 >> np.uint64(32)) + (p01 & lo32) + (p10 & lo32)
        return p11 + (p01 >> np.uint64(32)) + (p10 >> np.uint64(32)) + (mid >> np.uint64(32))


def bounded(x: np.ndarray, a: int, b: int) -> np.ndarray:
    """Lemire multiply-shift map of uint64 draws onto the integers [a, b]."""
    return mulhi64(x, b - a + 1).astype(np.int64) + np.int64(a)


def payload(seed: int, byte_off: int, nbytes: int) -> np.ndarray:
    """Bytes [byte_off, byte_off+nbytes) of the little-endian byte view of a stream."""
    if nbytes <= 0:
        return np.zeros(0, dtype=np.uint8)
    w0 = byte_off // 8
    w1 = (byte_off + nbytes + 7) // 8
    words = splitmix64(seed, w0, w1 - w0).astype("<u8")
    b = words.view(np.uint8)
    s = byte_off - w0 * 8
    return b[s:s + nbytes].copy()


def uniform_f32(x: np.ndarray) -> np.ndarray:
    """uniform[-1, 1) floats: ((x >> 40) * 2^-24) * 2 - 1, exact in fp32."""
    return ((x >> np.uint64(40)).astype(np.float64) * (2.0 ** -24) * 2.0 - 1.0).astype(np.float32)


def f32_to_bf16_bits(f: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even fp32 -> bf16, returned as uint16 bit patterns."""
    u = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))
    return ((u + rounding) >> np.uint64(16)).astype(np.uint16)


def unit_double(x: np.ndarray) -> np.ndarray:
    """53-bit uniform doubles in [0, 1)."""
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def derangement(seed: int, n: int) -> np.ndarray:
    """Fisher-Yates permutation of range(n) with no fixed point (resampled)."""
    if n < 2:
        raise ValueError("a derangement needs n >= 2")
    attempt = 0
    while True:
        x = splitmix64(seed, attempt * n, n)
        perm = np.arange(n, dtype=np.int64)
        for i in range(n - 1, 0, -1):
            j = int(bounded(x[i:i + 1], 0, i)[0])
            perm[i], perm[j] = perm[j], perm[i]
        if not np.any(perm == np.arange(n)):
            return perm
        attempt += 1


def ring(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.int64) + 1) % n


# ------------------------------------------------------- operation records
# Operation codes and descriptor layout shared by every consumer.  The values
# are part of the library's C-ABI (include/vshmem.h) and are repeated there.
OP_NOP = 0
OP_PUT = 1
OP_GET = 2
OP_PUT_SIGNAL = 3
OP_AMO_FETCH_ADD = 4
OP_AMO_FETCH_XOR = 5
OP_AMO_COMPARE_SWAP = 6
OP_AMO_ADD = 7
OP_AMO_XOR = 8
OP_AMO_SET = 9
OP_AMO_FETCH = 10
OP_AMO_SWAP = 11
OP_WAIT_UNTIL = 12
OP_FENCE = 13
OP_QUIET = 14
OP_BARRIER_ALL = 15

SCOPE_THREAD = 0
SCOPE_WAVE = 1
SCOPE_WG = 2
SCOPE_GRID = 3
SCOPE_AUTO = 255

SIGNAL_SET = 0
SIGNAL_ADD = 1

CMP_EQ, CMP_NE, CMP_GT, CMP_GE, CMP_LT, CMP_LE = range(6)

NO_RESULT = 0xFFFFFFFF

DESC_DTYPE = np.dtype([
    ("op", "u1"), ("scope", "u1"), ("aux", "u1"), ("flags", "u1"),
    ("issuer", "<i4"), ("target", "<i4"), ("result_idx", "<u4"),
    ("src", "<u8"), ("dst", "<u8"), ("nbytes", "<u8"),
    ("value", "<u8"), ("cond", "<u8"), ("reserved", "<u8"),
])
assert DESC_DTYPE.itemsize == 64


def descs(records: List[tuple]) -> np.ndarray:
    """Build a descriptor array from (op, scope, aux, issuer, target, result_idx,
    src, dst, nbytes, value, cond) tuples."""
    a = np.zeros(len(records), dtype=DESC_DTYPE)
    for i, r in enumerate(records):
        op, scope, aux, issuer, target, ridx, src, dst, n, value, cond = r
        a[i] = (op, scope, aux, 0, issuer, target, ridx, src, dst, n,
                value & _MASK64, cond & _MASK64, 0)
    return a


# ------------------------------------------------------------ heap filling
def heap_fill(base_seed: int, npes: int, nbytes: int) -> np.ndarray:
    """Initial contents of every PE's first ``nbytes`` bytes: (npes, nbytes) uint8."""
    out = np.empty((npes, nbytes), dtype=np.uint8)
    for p in range(npes):
        out[p] = payload(subseed(base_seed, TAG_HEAP + p), 0, nbytes)
    return out


# ------------------------------------------------- small mixed workload
@dataclasses.dataclass
class SmallWorkload:
    npes: int
    heap_bytes: int          # user bytes per PE
    data_bytes: int          # put/get area [0, data_bytes)
    counter_off: int         # 64 int64 counters live here on their home PE
    ncounters: int
    counter_home: np.ndarray
    descs: np.ndarray        # program: epochs separated by per-PE BARRIER_ALL
    n_rma: int
    n_amo: int
    init: np.ndarray         # (npes, heap_bytes) initial bytes


def _overlaps(iv: List[Tuple[int, int]], lo: int, hi: int) -> bool:
    for a, b in iv:
        if lo < b and a < hi:
            return True
    return False


def small_workload(seed: int = SEED_SMALL, npes: int = 4, heap_bytes: int = 1 << 20,
                   n_rma: int = 1000, epoch_ops: int = 125, n_amo: int = 10_000,
                   ncounters: int = 64, min_size: int = 8, max_size: int = 4096,
                   scope: int = SCOPE_AUTO, amo_scope: int = SCOPE_THREAD,
                   base_off: int = 0, fill: bool = True) -> SmallWorkload:
    """Mixed put/get traffic plus contended fetch_add on one small heap.

    The put/get ops are grouped into epochs of ``epoch_ops``; every epoch is
    conflict free (no byte written by one op is read or written by another op
    of that epoch) by rejection, and epochs are separated by barrier_all.
    The AMO epoch follows, then quiet and barrier_all.  All offsets are
    relative to ``base_off``: the workload occupies [base_off, base_off +
    heap_bytes) of every PE and ``init`` holds that window.
    """
    counter_off = heap_bytes - 4096
    data_bytes = counter_off
    if fill:
        init = heap_fill(seed, npes, heap_bytes)
        init[:, counter_off:counter_off + 8 * ncounters] = 0
    else:
        init = np.zeros((0, 0), dtype=np.uint8)
    rs = subseed(seed, TAG_OPS)
    ctr = 0

    def draw(k):
        nonlocal ctr
        x = splitmix64(rs, ctr, k)
        ctr += k
        return x

    recs = []
    made = 0
    while made < n_rma:
        nthis = min(epoch_ops, n_rma - made)
        writes = [[] for _ in range(npes)]
        reads = [[] for _ in range(npes)]
        k = 0
        while k < nthis:
            x = draw(6)
            kind = OP_PUT if (int(x[0]) & 1) == 0 else OP_GET
            issuer = int(bounded(x[1:2], 0, npes - 1)[0])
            target = int(bounded(x[2:3], 0, npes - 1)[0])
            n = int(bounded(x[3:4], min_size, max_size)[0])
            nslots = (data_bytes - n) // 8
            src = 8 * int(bounded(x[4:5], 0, nslots)[0])
            dst = 8 * int(bounded(x[5:6], 0, nslots)[0])
            if kind == OP_PUT:
                wpe, rpe = target, issuer
            else:
                wpe, rpe = issuer, target
            if wpe == rpe and src < dst + n and dst < src + n:
                continue
            if _overlaps(writes[wpe], dst, dst + n) or _overlaps(reads[wpe], dst, dst + n):
                continue
            if _overlaps(writes[rpe], src, src + n):
                continue
            writes[wpe].append((dst, dst + n))
            reads[rpe].append((src, src + n))
            recs.append((kind, scope, 0, issuer, target, NO_RESULT, base_off + src, base_off + dst, n, 0, 0))
            k += 1
        made += nthis
        for p in range(npes):
            recs.append((OP_BARRIER_ALL, SCOPE_WG, 0, p, p, NO_RESULT, 0, 0, 0, 0, 0))
    ra = subseed(seed, TAG_AMO)
    home = bounded(splitmix64(ra, 0, ncounters), 0, npes - 1)
    x = splitmix64(ra, ncounters, 2 * n_amo)
    issuers = bounded(x[0::2], 0, npes - 1)
    cidx = bounded(x[1::2], 0, ncounters - 1)
    for i in range(n_amo):
        c = int(cidx[i])
        recs.append((OP_AMO_FETCH_ADD, amo_scope, 0, int(issuers[i]), int(home[c]), i,
                     base_off + counter_off + 8 * c, 0, 8, 1, 0))
    for p in range(npes):
        recs.append((OP_QUIET, SCOPE_WG, 0, p, p, NO_RESULT, 0, 0, 0, 0, 0))
    for p in range(npes):
        recs.append((OP_BARRIER_ALL, SCOPE_WG, 0, p, p, NO_RESULT, 0, 0, 0, 0, 0))
    return SmallWorkload(npes, heap_bytes, data_bytes, counter_off, ncounters, home,
                         descs(recs), n_rma, n_amo, init)


# ------------------------------------------------------ bandwidth rounds
def sweep_sizes(lo_log2: int = 3, hi_log2: int = 26) -> List[int]:
    return [1 << k for k in range(lo_log2, hi_log2 + 1)]


def msgs_per_pe(size: int, total_log2: int = 28, cap_log2: int = 14) -> int:
    """Messages per PE in one round: min(2^total / size, 2^cap)."""
    return min((1 << total_log2) // size, 1 << cap_log2)


def pattern_targets(pattern: str, npes: int, seed: int = SEED_SWEEP) -> np.ndarray:
    if pattern == "ring":
        return ring(npes)
    if pattern == "perm":
        return derangement(subseed(seed, TAG_PERM), npes)
    raise ValueError(pattern)


# ------------------------------------------------------------- GUPS stream
def gups_updates(seed: int, start: int, count: int, log2_table: int, add_every: int = 5):
    """Updates start..start+count-1: (index, value, is_add).

    Update u draws x_{3u}, x_{3u+1}, x_{3u+2} from the op stream:
    index = x_{3u} & (2^log2_table - 1), value = x_{3u+1},
    op = add iff x_{3u+2} mod add_every == 0, xor otherwise.
    """
    x = splitmix64(subseed(seed, TAG_OPS), 3 * start, 3 * count)
    idx = x[0::3] & np.uint64((1 << log2_table) - 1)
    val = x[1::3]
    is_add = (x[2::3] % np.uint64(add_every)) == np.uint64(0)
    return idx, val, is_add


# ------------------------------------------------------------ collectives
def coll_f32(seed: int, pe: int, count: int) -> np.ndarray:
    return uniform_f32(splitmix64(subseed(seed, TAG_HEAP + pe), 0, count))


def coll_i64(seed: int, pe: int, count: int) -> np.ndarray:
    return splitmix64(subseed(seed, TAG_HEAP + pe), 0, count).view(np.int64)


def coll_bf16(seed: int, pe: int, count: int) -> np.ndarray:
    return f32_to_bf16_bits(coll_f32(seed, pe, count))


# Edge-case inputs of the reductions.  Column k of the (npes, count) array
# belongs to category k mod (number of categories); each element is a bit
# pattern drawn from its category's set with SplitMix64 draws.  The arrays
# are storage bits: int64 values, fp32 bits (uint32) or bf16 bits (uint16).
EDGE_I64_CATS = ("extremes", "min_max_only", "full_range", "equal")
EDGE_F32_CATS = ("signed_zeros", "subnormals", "subnormal_boundary", "one_inf", "both_infs",
                 "near_max", "nan", "mixed", "uniform")
EDGE_BF16_CATS = ("signed_zeros", "subnormals", "subnormal_boundary", "one_inf", "both_infs",
                  "near_max", "nan", "final_tie", "uniform")


def reduce_edge_columns(dt: int, npes: int, count: int, seed: int) -> np.ndarray:
    """dt: 0 int64, 1 fp32, 2 bf16 (the reductions' datatype codes)."""
    x = splitmix64(seed, 0, 4 * npes * count).reshape(npes, count, 4)
    a, b, c, d = (x[..., i] for i in range(4))
    col = np.arange(count)[None, :].repeat(npes, 0)
    pe = np.arange(npes)[:, None].repeat(count, 1)
    sign = (a >> np.uint64(63)).astype(np.uint64)
    # one position per column, for the categories that plant a special value
    pick = bounded(splitmix64(seed ^ 0x51, 0, count), 0, npes - 1)[None, :].repeat(npes, 0)
    pick2 = bounded(splitmix64(seed ^ 0x52, 0, count), 0, npes - 1)[None, :].repeat(npes, 0)
    if dt == 0:
        cat = col % len(EDGE_I64_CATS)
        ext = np.array([-(1 << 63), (1 << 63) - 1, -1, 0, 1, -(1 << 63) + 1, (1 << 63) - 2], dtype=np.int64)
        out = np.where(cat == 0, ext[bounded(b, 0, len(ext) - 1)], 0)
        out = np.where(cat == 1, np.where(sign == 1, ext[0], ext[1]), out)
        out = np.where(cat == 2, c.view(np.int64), out)
        out = np.where(cat == 3, (d[0:1, :].view(np.int64)).repeat(npes, 0), out)
        return out.astype(np.int64)
    if dt == 1:
        ncat = len(EDGE_F32_CATS)
        cat = col % ncat
        sbit = sign << np.uint64(31)
        uni = uniform_f32(b).view(np.uint32).astype(np.uint64)
        sub_small = sbit | np.maximum(c & np.uint64(0xFFFF), np.uint64(1))      # 0 < |x| < 2^-133
        sub_any = sbit | (c & np.uint64(0x7FFFFF))                              # any subnormal
        near_min = sbit | (bounded(d, 1, 2).astype(np.uint64) << np.uint64(23)) | (c & np.uint64(0x7FFFFF))
        near_max = sbit | np.uint64(0x7F7FFFFF) - (c & np.uint64(0xFFFF))
        qnan = np.uint64(0x7FC00000) | (c & np.uint64(0x3FFFFF)) | sbit
        inf = sbit | np.uint64(0x7F800000)
        out = np.zeros((npes, count), dtype=np.uint64)
        out = np.where(cat == 0, sbit, out)
        out = np.where(cat == 1, sub_small, out)
        out = np.where(cat == 2, np.where((d & np.uint64(1)) == 0, sub_any, near_min), out)
        out = np.where(cat == 3, np.where(pe == pick, inf, uni), out)
        out = np.where(cat == 4, np.where(pe == pick, np.uint64(0x7F800000),
                                          np.where(pe == (pick + 1) % npes, np.uint64(0xFF800000), uni)), out)
        out = np.where(cat == 5, near_max, out)
        out = np.where(cat == 6, np.where(pe == pick, qnan, uni), out)
        mix_set = np.stack([sbit, sub_any, near_min, uni, near_max, inf])
        out = np.where(cat == 7, np.take_along_axis(mix_set, bounded(d, 0, 5)[None].astype(np.int64), 0)[0], out)
        out = np.where(cat == 8, uni, out)
        return out.astype(np.uint32)
    ncat = len(EDGE_BF16_CATS)
    cat = col % ncat
    sbit = sign << np.uint64(15)
    uni = f32_to_bf16_bits(uniform_f32(b)).astype(np.uint64)
    sub = sbit | np.maximum(c & np.uint64(0x7F), np.uint64(1))
    near_min = sbit | (bounded(d, 1, 2).astype(np.uint64) << np.uint64(7)) | (c & np.uint64(0x7F))
    near_max = sbit | np.uint64(0x7F7F) - (c & np.uint64(0x3))
    inf = sbit | np.uint64(0x7F80)
    qnan = np.uint64(0x7FC0) | (c & np.uint64(0x3F)) | sbit
    # final_tie: a normal value at `pick` and, at `pick2`, half of its unit in
    # the last place (exponent 8 below, mantissa 0) with a random sign; every
    # other element a signed zero, so the fp32 sum lies halfway between two
    # bf16 values whenever pick != pick2.
    exp = bounded(d, 20, 200).astype(np.uint64)
    base_v = (exp << np.uint64(7)) | (c & np.uint64(0x7F))
    half = sbit | ((exp - np.uint64(8)) << np.uint64(7))
    out = np.zeros((npes, count), dtype=np.uint64)
    out = np.where(cat == 0, sbit, out)
    out = np.where(cat == 1, sub, out)
    out = np.where(cat == 2, np.where((d & np.uint64(1)) == 0, sub, near_min), out)
    out = np.where(cat == 3, np.where(pe == pick, inf, uni), out)
    out = np.where(cat == 4, np.where(pe == pick, np.uint64(0x7F80),
                                      np.where(pe == (pick + 1) % npes, np.uint64(0xFF80), uni)), out)
    out = np.where(cat == 5, near_max, out)
    out = np.where(cat == 6, np.where(pe == pick, qnan, uni), out)
    out = np.where(cat == 7, np.where(pe == pick, base_v, np.where(pe == pick2, half, sbit)), out)
    out = np.where(cat == 8, uni, out)
    return out.astype(np.uint16)


# --------------------------------------------------------------- serving
@dataclasses.dataclass
class ServeRequest:
    kind: int          # OP_PUT / OP_GET / OP_AMO_FETCH_ADD
    issuer: int
    target: int
    nbytes: int
    arrival_s: float
    lane: int


def serve_requests(seed: int, n: int, npes: int, rate_per_s: float, lanes: int = 8,
                   min_size: int = 64, size_log2_span: int = 18) -> List[ServeRequest]:
    """Poisson arrivals over ``lanes`` lanes; sizes floor(64 * 2^(18u)) bytes
    (log-uniform 64 B - 16 MiB); kind uniform over put/get/fetch_add; issuer
    and target uniform over the PEs."""
    xs = splitmix64(subseed(seed, TAG_SIZES), 0, 5 * n)
    xa = splitmix64(subseed(seed, TAG_ARRIVAL), 0, n)
    u = unit_double(xs[0::5])
    sizes = np.floor(min_size * np.exp2(size_log2_span * u)).astype(np.int64)
    kinds = bounded(xs[1::5], 0, 2)
    issuer = bounded(xs[2::5], 0, npes - 1)
    target = bounded(xs[3::5], 0, npes - 1)
    lane = bounded(xs[4::5], 0, lanes - 1)
    gaps = -np.log1p(-unit_double(xa)) / rate_per_s
    t = np.cumsum(gaps)
    kind_map = [OP_PUT, OP_GET, OP_AMO_FETCH_ADD]
    out = []
    for i in range(n):
        nb = int(sizes[i])
        k = kind_map[int(kinds[i])]
        if k == OP_AMO_FETCH_ADD:
            nb = max(8, nb & ~7)
        out.append(ServeRequest(k, int(issuer[i]), int(target[i]), nb, float(t[i]), int(lane[i])))
    return out


def log2_class(n: int) -> int:
    return max(0, int(math.floor(math.log2(max(1, n)))))
