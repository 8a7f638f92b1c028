"""Seeded synthetic inputs for CP decomposition workloads.

This module only draws random numbers and builds planted tensors from factor
matrices; it holds none of the decomposition's arithmetic.  It is the one
piece of code that both the GPU path's callers (tests, benchmark) and the CPU
oracle's callers use, so that both sides see the same inputs.

Recipe (every workload):
  * SeedSequence(seed).spawn(3) gives three independent streams: planted
    factors, noise, initial factors.
  * Planted factors are drawn mode by mode, one (s_n, R) array per mode.
  * The noiseless tensor T0 = sum_r a^(0)_r o ... o a^(N-1)_r is built in FP64,
    in row blocks of the first mode.
  * Noise is iid Gaussian with sigma = rel * ||T0||_F / sqrt(numel), drawn in
    the same row blocks (one standard_normal call per block, in order), so
    that ||E||_F is close to rel * ||T0||_F.
  * The stored tensor is (T0 + sigma * E) cast to the storage dtype; with
    nonneg=True it is clipped at zero first (non-negative data).
  * Initial factors are iid Uniform[0, 1) (the paper's initialization).

Factor distributions:
  "uniform"   iid Uniform[0, 1)
  "lognorm"   iid N(0, 1) columns, normalized, scaled by 10**Uniform(-2, 0)
  "collinear" per factor: g, z_r ~ N(0, I); column r = sqrt(c) g + sqrt(1-c) z_r,
              then normalized (expected pairwise cosine close to c)
  "normal"    iid N(0, 1)
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Workload:
    name: str
    dims: tuple
    R: int
    T: np.ndarray          # stored tensor (storage dtype), C order
    planted: list          # FP64 planted factors
    init: list             # FP64 initial factors
    sigma: float
    norm_T0: float


def _factors(rng, dims, R, kind, collinearity=0.9):
    out = []
    for s in dims:
        if kind == "uniform":
            A = rng.random((s, R))
        elif kind == "normal":
            A = rng.standard_normal((s, R))
        elif kind == "lognorm":
            A = rng.standard_normal((s, R))
            A /= np.linalg.norm(A, axis=0, keepdims=True)
            A *= 10.0 ** rng.uniform(-2.0, 0.0, size=R)[None, :]
        elif kind == "collinear":
            g = rng.standard_normal(s)
            Z = rng.standard_normal((s, R))
            A = np.sqrt(collinearity) * g[:, None] + np.sqrt(1.0 - collinearity) * Z
            A /= np.linalg.norm(A, axis=0, keepdims=True)
        else:
            raise ValueError(kind)
        out.append(A)
    return out


def _outer_rows(factors, rows):
    """Rows `rows` of the first mode of the planted tensor, FP64, flattened."""
    K = factors[1]
    for F in factors[2:]:
        K = (K[:, None, :] * F[None, :, :]).reshape(K.shape[0] * F.shape[0], K.shape[1])
    return factors[0][rows] @ K.T


def planted_tensor(dims, R, seed, kind="uniform", noise_rel=1e-2, dtype=np.float32,
                   collinearity=0.9, block_elems=1 << 24, name="custom", nonneg=False):
    dims = tuple(int(d) for d in dims)
    rng_p, rng_e, rng_i = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3)]
    planted = _factors(rng_p, dims, R, kind, collinearity)
    init = [rng_i.random((s, R)) for s in dims]
    rest = int(np.prod(dims[1:], dtype=np.int64))
    K = planted[1]
    for F in planted[2:]:
        K = (K[:, None, :] * F[None, :, :]).reshape(K.shape[0] * F.shape[0], K.shape[1])
    KT = np.ascontiguousarray(K.T)
    rows_per_block = max(1, block_elems // rest)
    T0 = np.empty((dims[0], rest), dtype=np.float64)
    nrm2 = 0.0
    for r0 in range(0, dims[0], rows_per_block):
        blk = planted[0][r0:r0 + rows_per_block] @ KT
        T0[r0:r0 + rows_per_block] = blk
        nrm2 += float(np.sum(blk * blk))
    del K, KT
    norm_T0 = float(np.sqrt(nrm2))
    numel = dims[0] * rest
    sigma = noise_rel * norm_T0 / np.sqrt(numel) if noise_rel > 0 else 0.0
    out = np.empty((dims[0], rest), dtype=dtype)
    for r0 in range(0, dims[0], rows_per_block):
        blk = T0[r0:r0 + rows_per_block]
        if sigma > 0:
            blk = blk + sigma * rng_e.standard_normal(blk.shape)
        if nonneg:
            blk = np.maximum(blk, 0.0)
        out[r0:r0 + rows_per_block] = blk.astype(dtype)
    del T0
    return Workload(name=name, dims=dims, R=R, T=out.reshape(dims), planted=planted, init=init,
                    sigma=sigma, norm_T0=norm_T0)


# Named workloads.  "small" variants keep each workload's structure (order,
# factor distribution, noise level, storage precision) at sizes the FP64
# oracle handles in seconds while still spanning several GPU tiles and a
# ragged tail.
WORKLOADS = {
    # order-3 64^3 FP64, planted rank 16 uniform, noise 1e-3, R = 16
    "o3_s64_r16_f64": dict(dims=(64, 64, 64), R=16, seed=1001, kind="uniform", noise_rel=1e-3,
                           dtype=np.float64),
    # order-4 128^4 FP32, planted rank 64 uniform, noise 1e-2, R = 64
    "o4_s128_r64_f32": dict(dims=(128, 128, 128, 128), R=64, seed=2001, kind="uniform",
                            noise_rel=1e-2, dtype=np.float32),
    # order-6 24^6 FP32, planted rank 32 collinear (0.9), noise 1e-2, R = 32
    "o6_s24_r32_f32_col": dict(dims=(24,) * 6, R=32, seed=4001, kind="collinear", noise_rel=1e-2,
                               dtype=np.float32),
    # reduced shapes of the same families
    "o4_small_f32": dict(dims=(40, 37, 33, 29), R=20, seed=2002, kind="uniform", noise_rel=1e-2,
                         dtype=np.float32),
    "o3_small_f64": dict(dims=(37, 45, 29), R=12, seed=1002, kind="uniform", noise_rel=1e-3,
                         dtype=np.float64),
    # rank above 64 (the R x R operands split into two 64-column chunks) and a
    # long mode (several 16-row blocks per workgroup of a mode update)
    "o3_r80_f64": dict(dims=(200, 40, 36), R=80, seed=1003, kind="normal", noise_rel=1e-3,
                       dtype=np.float64),
    "o3_r40_long_f64": dict(dims=(1400, 12, 10), R=40, seed=1004, kind="normal", noise_rel=1e-3,
                            dtype=np.float64),
    # orders 5 and 6 (the PP dimension tree's levels 3 and 4, five or more
    # pair corrections per mode, the multi-pair bracket of Eq. (7)), FP64
    "o5_small_f64": dict(dims=(9, 8, 7, 6, 5), R=6, seed=5101, kind="uniform", noise_rel=1e-3,
                         dtype=np.float64),
    "o6_small_f64": dict(dims=(7, 8, 6, 9, 5, 6), R=8, seed=5103, kind="uniform", noise_rel=1e-3,
                         dtype=np.float64),
    # the order-6 collinear family at an oracle-sized shape
    "o6_col_small_f64": dict(dims=(10,) * 6, R=8, seed=4201, kind="collinear", noise_rel=1e-2,
                             dtype=np.float64),
    # Shape-only stand-ins for the paper's real tensors (the data themselves
    # are not available): the shapes and CP ranks of its experiments, planted
    # non-negative rank-R factors (Uniform[0, 1)), noise 1e-2, clipped at zero.
    # The density-fitting tensor is run at R = 128, the largest rank this
    # implementation supports (the paper uses 300, 600 and 1000).
    "coil_standin": dict(dims=(128, 128, 3, 7200), R=20, seed=6001, kind="uniform", noise_rel=1e-2,
                         dtype=np.float32, nonneg=True),
    "timelapse_standin": dict(dims=(1024, 1344, 33, 9), R=50, seed=6002, kind="uniform",
                              noise_rel=1e-2, dtype=np.float32, nonneg=True),
    "chem_standin": dict(dims=(4520, 280, 280), R=128, seed=6003, kind="uniform", noise_rel=1e-2,
                         dtype=np.float32, nonneg=True),
    # the same mode-size structure at oracle-sized shapes
    "coil_small": dict(dims=(32, 32, 3, 450), R=20, seed=6101, kind="uniform", noise_rel=1e-2,
                       dtype=np.float64, nonneg=True),
    "timelapse_small": dict(dims=(64, 84, 33, 9), R=50, seed=6102, kind="uniform", noise_rel=1e-2,
                            dtype=np.float64, nonneg=True),
    "chem_small": dict(dims=(565, 35, 35), R=64, seed=6103, kind="uniform", noise_rel=1e-2,
                       dtype=np.float64, nonneg=True),
}


def workload(name, **over):
    cfg = dict(WORKLOADS[name])
    cfg.update(over)
    return planted_tensor(name=name, **cfg)


def bf16_bits(x):
    """Round FP32 values to BF16 (nearest, ties to even); returns the raw
    16-bit patterns (uint16).  Storage conversion of a generated tensor."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_to_f32(bits):
    """The FP32 values of raw BF16 patterns (exact)."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


FP8_MAX = 448.0  # largest finite E4M3 value, 1.75 * 2^8


def _fp8_table():
    """The 256 E4M3 values: sign bit, 4-bit exponent with bias 7, 3-bit
    mantissa; exponent 0 holds the subnormals m 2^-9; exponent 15 with
    mantissa 7 is NaN (there are no infinities)."""
    b = np.arange(256, dtype=np.int64)
    e, m = (b >> 3) & 15, b & 7
    mag = np.where(e > 0, np.ldexp(8.0 + m, e - 10), np.ldexp(m.astype(np.float64), -9))
    v = np.where((b & 0x80) != 0, -mag, mag)
    return np.where((e == 15) & (m == 7), np.nan, v).astype(np.float32)


_FP8_VALUES = _fp8_table()


def fp8_to_f32(bits):
    """The FP32 values of raw FP8 E4M3 patterns (exact)."""
    return _FP8_VALUES[np.asarray(bits, dtype=np.uint8)]


def fp8_scale(x):
    """The largest power of two s with max |x| s <= FP8_MAX: the tensor times
    s uses E4M3's range (17 binades down to the subnormals) from the top.
    Scaling by a power of two is exact, and the relative residual of a CP
    fit does not depend on the tensor's scale."""
    m = float(np.max(np.abs(x)))
    if not np.isfinite(m) or m == 0.0:
        return 1.0
    s = 2.0 ** np.floor(np.log2(FP8_MAX / m))
    while m * s > FP8_MAX:  # guard the logarithm's rounding
        s /= 2
    return float(s)


def fp8_bits(x, scale=1.0, block=1 << 26):
    """Round FP32 values (times `scale`, a power of two, applied exactly) to
    FP8 E4M3 (nearest, ties to even); returns the raw 8-bit patterns (uint8).  Non-finite values, and values whose rounding
    exceeds FP8_MAX, are rejected.  Storage conversion of a generated
    tensor.  From 2^-6 up the FP32 pattern keeps its top 3 mantissa bits
    (rounded; a carry moves to the next binade) and its exponent is rebased
    from bias 127 to 7; below, the value is a multiple of 2^-9 (subnormals)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    flat = x.reshape(-1)
    out = np.empty(flat.shape, dtype=np.uint8)
    for s0 in range(0, flat.size, block):
        xs = flat[s0:s0 + block]
        if scale != 1.0:
            xs = xs * np.float32(scale)
        u = xs.view(np.uint32)
        a = u & np.uint32(0x7FFFFFFF)
        r = (a + np.uint32(0x7FFFF) + ((a >> np.uint32(20)) & np.uint32(1))) >> np.uint32(20)
        with np.errstate(over="ignore", invalid="ignore"):  # large or non-finite inputs take the other branch
            sub = np.rint(np.minimum(a.view(np.float32) * np.float32(512.0), np.float32(8.0))).astype(np.int32)
        code = np.where(a >= np.uint32(0x3C800000), r.astype(np.int32) - 960, sub)
        if code.size and code.max() > 0x7E:  # infinities and NaN land here too
            raise ValueError("fp8_bits: non-finite value or value beyond the E4M3 range")
        out[s0:s0 + block] = (code | ((u >> np.uint32(24)) & np.uint32(0x80)).astype(np.int32)).astype(np.uint8)
    return out.reshape(x.shape)



def batch_workload(count=512, seed=5001, smin=16, smax=96, ranks=(4, 8, 16, 32), noise_rel=1e-3):
    """Many small independent order-3 FP32 tensors: each mode size iid
    uniform on [smin, smax], rank uniform over `ranks`, planted iid
    Uniform[0, 1) factors plus Gaussian noise at `noise_rel` of the norm,
    initial factors iid Uniform[0, 1).  Tensor i uses seed
    SeedSequence(seed).spawn(count + 1)[i + 1] through planted_tensor; the
    first child draws the shapes."""
    children = np.random.SeedSequence(seed).spawn(count + 1)
    rng = np.random.default_rng(children[0])
    dims = rng.integers(smin, smax + 1, size=(count, 3))
    rs = rng.choice(np.asarray(ranks), size=count)
    out = []
    for i in range(count):
        s = int(children[i + 1].generate_state(1)[0])
        out.append(planted_tensor(tuple(int(x) for x in dims[i]), int(rs[i]), s, kind="uniform",
                                  noise_rel=noise_rel, dtype=np.float32, name=f"batch{i}"))
    return out
