"""User-defined reductions used by the tests: each case is the user's code
twice, as C++ text for omprt_udr_declare and as Python for the oracle's
sequential fold (oracle.udr_fold).  Both are inputs to the two sides; the
oracle pins check the Python versions against independent computations.

* WELFORD (fp32 / bf16 / fp64 input): count, mean and M2 with Welford's
  update per element and Chan et al.'s pairwise combination, in double.
* STATS3 (int32 input): multiples of 3, sum of squares modulo 2^64, XOR of a
  position hash -- exact.
* MINMAX (fp64 input): minimum with its first position, and the maximum --
  exact.
* HIST16 (int64 input): a 16-bin histogram of the low four bits, 64 bytes,
  the largest type (four cross-team slots) -- exact.
* SUMSQ (bf16 input): sum of squares in double.
"""
import struct

import numpy as np

M64 = (1 << 64) - 1
GOLD = 0x9E3779B97F4A7C15

WELFORD = dict(
    type_def="struct omp_type { double n, mean, m2; };",
    initializer="omp_priv = omp_type{0.0, 0.0, 0.0};",
    combiner="""
        const double n = omp_out.n + omp_in.n;
        if (n > 0) {
            const double d = omp_in.mean - omp_out.mean;
            omp_out.mean += d * (omp_in.n / n);
            omp_out.m2 += omp_in.m2 + d * d * (omp_out.n * omp_in.n / n);
            omp_out.n = n;
        }""",
    body="""
        const double v = omp_elem;
        omp_priv.n += 1.0;
        const double d = v - omp_priv.mean;
        omp_priv.mean += d / omp_priv.n;
        omp_priv.m2 += d * (v - omp_priv.mean);""",
    acc_bytes=24)


def welford_init():
    return (0.0, 0.0, 0.0)


def welford_body(p, v, i):
    n, mean, m2 = p
    n += 1.0
    d = float(v) - mean
    mean += d / n
    return (n, mean, m2 + d * (float(v) - mean))


def welford_combine(o, i):
    n = o[0] + i[0]
    if n <= 0:
        return o
    d = i[1] - o[1]
    return (n, o[1] + d * (i[0] / n), o[2] + i[2] + d * d * (o[0] * i[0] / n))


STATS3 = dict(
    type_def="struct omp_type { uint64_t cnt3, sq, h; };",
    initializer="omp_priv = omp_type{0, 0, 0};",
    combiner="omp_out.cnt3 += omp_in.cnt3; omp_out.sq += omp_in.sq; omp_out.h ^= omp_in.h;",
    body="""
        if (omp_elem % 3 == 0) omp_priv.cnt3 += 1;
        omp_priv.sq += (uint64_t)((int64_t)omp_elem * (int64_t)omp_elem);
        omp_priv.h ^= ((uint64_t)(omp_i + 1) * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(uint32_t)omp_elem;""",
    acc_bytes=24)


def stats3_init():
    return (0, 0, 0)


def stats3_body(p, v, i):
    v = int(v)
    return (p[0] + (1 if v % 3 == 0 else 0), (p[1] + v * v) & M64,
            p[2] ^ ((((i + 1) * GOLD) & M64) ^ (v & 0xFFFFFFFF)))


def stats3_combine(o, i):
    return (o[0] + i[0], (o[1] + i[1]) & M64, o[2] ^ i[2])


MINMAX = dict(
    type_def="struct omp_type { double mn, mx; int64_t imn; int64_t pad; };",
    initializer="omp_priv = omp_type{__builtin_huge_val(), -__builtin_huge_val(), INT64_MAX, 0};",
    combiner="""
        if (omp_in.mn < omp_out.mn || (omp_in.mn == omp_out.mn && omp_in.imn < omp_out.imn)) {
            omp_out.mn = omp_in.mn;
            omp_out.imn = omp_in.imn;
        }
        if (omp_in.mx > omp_out.mx) omp_out.mx = omp_in.mx;""",
    body="""
        if (omp_elem < omp_priv.mn) { omp_priv.mn = omp_elem; omp_priv.imn = omp_i; }
        if (omp_elem > omp_priv.mx) omp_priv.mx = omp_elem;""",
    acc_bytes=32)


def minmax_init():
    return (float("inf"), float("-inf"), (1 << 63) - 1, 0)


def minmax_body(p, v, i):
    mn, mx, imn, pad = p
    v = float(v)
    if v < mn:
        mn, imn = v, i
    return (mn, max(mx, v), imn, pad)


def minmax_combine(o, i):
    mn, mx, imn, pad = o
    if i[0] < mn or (i[0] == mn and i[2] < imn):
        mn, imn = i[0], i[2]
    return (mn, max(mx, i[1]), imn, pad)


HIST16 = dict(
    type_def="struct omp_type { uint32_t bin[16]; };",
    initializer="for (int b = 0; b < 16; ++b) omp_priv.bin[b] = 0;",
    combiner="for (int b = 0; b < 16; ++b) omp_out.bin[b] += omp_in.bin[b];",
    body="omp_priv.bin[omp_elem & 15] += 1;",
    acc_bytes=64)


def hist16_init():
    return tuple([0] * 16)


def hist16_body(p, v, i):
    q = list(p)
    q[int(v) & 15] = (q[int(v) & 15] + 1) & 0xFFFFFFFF
    return tuple(q)


def hist16_combine(o, i):
    return tuple((a + b) & 0xFFFFFFFF for a, b in zip(o, i))


SUMSQ = dict(
    type_def="struct omp_type { double s; };",
    initializer="omp_priv.s = 0.0;",
    combiner="omp_out.s += omp_in.s;",
    body="omp_priv.s += (double)omp_elem * (double)omp_elem;",
    acc_bytes=8)


def sumsq_init():
    return (0.0,)


def sumsq_body(p, v, i):
    return (p[0] + float(v) * float(v),)


def sumsq_combine(o, i):
    return (o[0] + i[0],)


# packing of omp_type values as bytes (for device tensors)
FORMATS = {"WELFORD": "<3d", "STATS3": "<3Q", "MINMAX": "<2d2q", "HIST16": "<16I", "SUMSQ": "<d"}


def pack(name, value):
    return np.frombuffer(struct.pack(FORMATS[name], *value), dtype=np.uint8).copy()


def unpack(name, raw):
    return struct.unpack(FORMATS[name], bytes(np.asarray(raw, dtype=np.uint8)))
