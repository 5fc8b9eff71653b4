"""Device primitives of the gbest aggregation (Alg. 1 Step 5, in the place
of the queue of Sec. 3.1 Alg. 2 and the lock of Sec. 3.2 Alg. 3), run on the
GPU through test kernels around the library's own device functions and
checked against brute force: the packed (fitness, index) key, the wavefront
minimum, the workgroup minimum of the keys below a threshold, the
device-wide 64-bit atomicMin publish, and the seqlock of the asynchronous
variant under concurrent writers and readers.

Adversarial cases: every key tied, a lone candidate in lane 63, every lane a
candidate, NaN fitness, the no-candidate sentinel, thresholds equal to a key."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hip", "libpso_prims.so")
NO_KEY = np.uint64(2**64 - 1)
U64 = np.uint64

_lib = None


def prims():
    global _lib
    if _lib is None:
        from paper_2205_01313_amd import _native

        _native._single_hip_runtime()  # the HIP runtime torch loaded, as libpso uses
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run tests/hip/build_prims.py")
        lib = ctypes.CDLL(LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.prim_make_key.argtypes = [vp, vp, i64, vp]
        lib.prim_wave_min.argtypes = [vp, i64, vp]
        lib.prim_group_min.argtypes = [vp, vp, i64, i32, vp]
        lib.prim_publish_sync.argtypes = [vp, i64, ctypes.c_uint64, ctypes.c_uint64, vp]
        lib.prim_seqlock_stress.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp]
        lib.prim_philox_rate.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, i64, vp, vp]
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def dev_keys(f, idx):
    f = np.ascontiguousarray(f, np.float32)
    idx = np.ascontiguousarray(idx, np.uint32)
    out = np.empty(len(f), np.uint64)
    assert prims().prim_make_key(_p(f), _p(idx), len(f), _p(out)) == 0
    return out


def wave_min(vals):
    vals = np.ascontiguousarray(vals, np.uint64)
    assert vals.size % 64 == 0
    out = np.empty_like(vals)
    assert prims().prim_wave_min(_p(vals), vals.size // 64, _p(out)) == 0
    return out.reshape(-1, 64)


def group_min(keys, thr, lanes):
    keys = np.ascontiguousarray(keys, np.uint64)
    thr = np.ascontiguousarray(thr, np.uint64)
    groups = keys.size // lanes
    out = np.empty_like(keys)
    assert prims().prim_group_min(_p(keys), _p(thr), groups, lanes, _p(out)) == 0
    return out.reshape(groups, lanes)


def brute_group_min(keys, thr):
    cand = keys < thr
    return keys[cand].min() if cand.any() else NO_KEY


def key_of(order_hi, idx):
    return U64((int(order_hi) << 32) | int(idx))


# ---------------------------------------------------------------------------
# packed key
# ---------------------------------------------------------------------------
def test_make_key_equals_oracle_key_on_special_values():
    announce("prims: make_key vs the oracle's key over special and random values")
    rng = np.random.default_rng(0)
    special = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, -np.nan, 1e-45, -1e-45, 1.1754942e-38,
                        3.4028235e38, -3.4028235e38, 5e-324], np.float32)
    f = np.concatenate([special, rng.standard_normal(4000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 4000)])
    f = f.astype(np.float32)
    idx = rng.integers(0, 2**32, f.size, dtype=np.uint64).astype(np.uint32)
    idx[:3] = [0, 0xFFFFFFFF, 7]
    got = dev_keys(f, idx)
    want = oracle.keys(f, idx)
    assert np.array_equal(got, want)
    # +0 and -0 share a key; a NaN's order bits are the largest
    assert got[0] >> U64(32) == got[1] >> U64(32)
    assert (got[6] >> U64(32)) == U64(0xFFFFFFFF) and (got[7] >> U64(32)) == U64(0xFFFFFFFF)
    # key order equals (fitness, index) order wherever neither is NaN
    ok = ~np.isnan(f)
    o = np.lexsort((idx[ok], f[ok].astype(np.float64)))
    assert np.all(np.diff(got[ok][o].astype(object)) >= 0)


# ---------------------------------------------------------------------------
# wavefront minimum
# ---------------------------------------------------------------------------
def test_wave_min_adversarial():
    announce("prims: wave_min_u64 on tied, lone-lane, all-lane, sentinel and random wavefronts")
    rng = np.random.default_rng(1)
    waves = []
    waves.append(np.full(64, key_of(0x80000000, 5), np.uint64))                # every lane tied
    w = np.full(64, NO_KEY, np.uint64); w[63] = key_of(0x3F800000 | 0x80000000, 9); waves.append(w)  # lone lane 63
    w = np.full(64, NO_KEY, np.uint64); w[0] = key_of(0xBF800000, 1); waves.append(w)                # lone lane 0
    waves.append(np.full(64, NO_KEY, np.uint64))                                # nothing
    waves.append(np.arange(64, dtype=np.uint64)[::-1].copy() + U64(1 << 40))   # every lane distinct, min at 63
    w = np.full(64, key_of(0xFFFFFFFF, 3), np.uint64); w[17] = key_of(0xFFFFFFFF, 2); waves.append(w)  # NaN keys
    w = np.full(64, key_of(0xC0000000, 100), np.uint64); w[::2] = key_of(0xC0000000, 99); waves.append(w)  # ties by fitness
    for _ in range(64):
        waves.append(rng.integers(0, 2**64 - 1, 64, dtype=np.uint64))
    # keys differing only in the low word or only in bit 63
    w = rng.integers(0, 2**32, 64, dtype=np.uint64) | U64(0xABCD0000 << 32); waves.append(w)
    w = np.full(64, U64(1 << 63), np.uint64); w[40] = U64((1 << 63) - 1); waves.append(w)
    vals = np.concatenate(waves)
    out = wave_min(vals)
    for k, w in enumerate(waves):
        assert np.all(out[k] == w.min()), (k, out[k][:4], w.min())


# ---------------------------------------------------------------------------
# workgroup minimum with the candidate filter
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lanes", [64, 256, 1024])
def test_group_min_adversarial(lanes):
    announce(f"prims: workgroup_min at {lanes} lanes against brute force")
    rng = np.random.default_rng(2 + lanes)
    groups, thrs = [], []

    def add(keys, thr):
        groups.append(np.asarray(keys, np.uint64))
        thrs.append(U64(thr))

    base = key_of(0x90000000, 0)
    add(np.full(lanes, base, np.uint64), NO_KEY)                       # every lane tied, all candidates
    add(np.full(lanes, base, np.uint64), base)                         # tied and equal to the threshold: none
    k = np.full(lanes, NO_KEY, np.uint64); k[63] = base; add(k, NO_KEY)  # lone candidate in lane 63
    k = np.full(lanes, NO_KEY, np.uint64); k[lanes - 1] = base; add(k, NO_KEY)  # lone candidate in the last lane
    k = np.arange(lanes, dtype=np.uint64) + base; add(k, base + U64(lanes))  # every lane a candidate
    k = np.arange(lanes, dtype=np.uint64) + base; add(k, base + U64(1))  # only lane 0 below the threshold
    k = np.full(lanes, key_of(0xFFFFFFFF, 4), np.uint64); add(k, NO_KEY)  # NaN fitness everywhere
    k = np.full(lanes, key_of(0xFFFFFFFF, 4), np.uint64); k[5] = base; add(k, key_of(0xFFFFFFFF, 0))  # NaN never a candidate below
    add(np.full(lanes, NO_KEY, np.uint64), NO_KEY)                     # the sentinel only
    for _ in range(40):
        k = rng.integers(0, 2**64 - 1, lanes, dtype=np.uint64)
        add(k, k[rng.integers(0, lanes)])                               # threshold equal to some lane's key
    for _ in range(20):
        k = rng.integers(2**62, 2**62 + 4, lanes, dtype=np.uint64)      # heavy ties
        add(k, U64(2**62 + 2))
    out = group_min(np.concatenate(groups), np.array(thrs, np.uint64), lanes)
    for g, (k, t) in enumerate(zip(groups, thrs)):
        want = brute_group_min(k, t)
        assert np.all(out[g] == want), (g, out[g][0], want)


# ---------------------------------------------------------------------------
# device-wide publish (packed-key atomicMin)
# ---------------------------------------------------------------------------
def test_publish_sync_reaches_the_minimum():
    announce("prims: publish_sync from many workgroups")
    rng = np.random.default_rng(3)
    lib = prims()
    out = np.zeros(1, np.uint64)
    for case in range(6):
        n = [1, 7, 1024, 4096, 4096, 2048][case]
        keys = rng.integers(0, 2**64 - 1, n, dtype=np.uint64)
        if case == 4:
            keys[:] = keys[0]                                            # every workgroup tied
        if case == 5:
            keys[:] = NO_KEY
            keys[-1] = U64(12345)                                        # the last workgroup alone
        thr = NO_KEY
        init = NO_KEY
        assert lib.prim_publish_sync(_p(keys), n, int(thr), int(init), _p(out)) == 0
        assert out[0] == keys.min(), case
    # keys not below the threshold are not published; a running key lower
    # than every candidate stays
    keys = rng.integers(1 << 40, 1 << 41, 512, dtype=np.uint64)
    thr = np.sort(keys)[100]
    assert lib.prim_publish_sync(_p(keys), keys.size, int(thr), int(NO_KEY), _p(out)) == 0
    assert out[0] == keys.min()
    assert lib.prim_publish_sync(_p(keys), keys.size, int(NO_KEY), 5, _p(out)) == 0
    assert out[0] == U64(5)
    keys2 = np.full(64, U64(1 << 50), np.uint64)
    assert lib.prim_publish_sync(_p(keys2), 64, int(U64(1 << 50)), int(NO_KEY), _p(out)) == 0
    assert out[0] == NO_KEY  # equal to the threshold: not a candidate


# ---------------------------------------------------------------------------
# seqlock under concurrent writers and readers
# ---------------------------------------------------------------------------
# Writers publishing back to back starve a reader of a wide position (its
# snapshot outlasts the gap between publishes, so it only completes once the
# writers stop); the widest case pauses the writers between publishes.
@pytest.mark.parametrize("D,writers,readers,rounds,gap",
                         [(32, 8, 24, 200, 0), (512, 16, 48, 100, 0), (4096, 4, 16, 50, 40)])
def test_seqlock_snapshots_never_torn(D, writers, readers, rounds, gap):
    announce(f"prims: seqlock stress D={D} writers={writers} readers={readers} rounds={rounds} gap={gap}")
    stats = np.zeros(5, np.uint32)
    key = np.zeros(1, np.uint64)
    pos = np.zeros(D, np.float32)
    assert prims().prim_seqlock_stress(D, writers, readers, rounds, gap, 200000, _p(stats), _p(key), _p(pos)) == 0
    torn, snaps, changes, err, done = (int(v) for v in stats)
    assert err == 0, "a bounded seqlock wait gave up"
    assert done == writers
    assert torn == 0, f"{torn} torn elements in {snaps} snapshots"
    assert snaps >= readers
    # readers saw publishes happen while they read (the run is concurrent)
    assert changes > readers, (changes, snaps)
    # the last publish is the smallest key: writer w, last round
    last = rounds * writers - 1
    want = U64(((0x90000000 - last) << 32) | last)
    assert key[0] == want
    assert np.array_equal(pos, (last * 4096 + np.arange(D)).astype(np.float32))


# ---------------------------------------------------------------------------
# random-number throughput
# ---------------------------------------------------------------------------
def test_philox_throughput_draws_equal_oracle():
    """The VALU cost of Philox4x32-10 (the step kernels' largest share of
    vector instructions): 2^20 lanes draw 256 blocks each with the step
    kernels' counter layout; sampled lanes' XOR of all draws equals the
    oracle's generator, and the rate is printed (draws per second and SIMD
    cycles per draw of one wavefront at 2.4 GHz over 1024 SIMDs) for the
    rocprofv3 counter pass that prices its instructions."""
    lanes, calls, k0, k1 = 1 << 20, 256, 0x01234567, 0x89ABCDEF
    announce(f"philox throughput: {lanes} lanes x {calls} draws")
    out = np.empty(lanes, np.uint32)
    ms = ctypes.c_float()
    assert prims().prim_philox_rate(k0, k1, calls, lanes, _p(out), ctypes.byref(ms)) == 0
    rng = np.random.default_rng(5)
    for lane in [0, 63, lanes - 1] + [int(x) for x in rng.integers(0, lanes, 5)]:
        acc = 0
        for j in range(calls):
            w = oracle.philox((k0, k1), (j, lane, 0, 0))
            acc ^= int(w[0]) ^ int(w[1]) ^ int(w[2]) ^ int(w[3])
        assert int(out[lane]) == acc, lane
    draws = lanes * calls
    cycles = ms.value * 1e-3 * 2.4e9 * 1024 / (draws / 64)
    print(f"\n{draws / (ms.value * 1e-3):.4g} draws/s; {cycles:.0f} SIMD cycles per wavefront draw ({ms.value:.3f} ms)")
