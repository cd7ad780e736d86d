"""Pins for the CPU oracle: each test checks it against something other than
itself -- Python's complex type, numpy's complex matmul, the paper's own Eq. 3
route, closed forms and invariants -- chosen so that a dropped term, a wrong
sign, a swapped index or a wrong offset fails at least one of them."""
import json
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def parts(f, t, n, seed, sigma=2.5, common=0.0):
    x, qr, qi = synth.quantized_gaussian(f, t, n, sigma, seed, common=common, return_parts=True)
    return x.numpy(), qr.numpy().astype(np.int64), qi.numpy().astype(np.int64)


def upper(full):
    """[F][N][N][2] -> packed row-major upper triangle [F][E][2] (numpy's order)."""
    n = full.shape[1]
    i, j = np.triu_indices(n)
    return full[:, i, j, :]


@pytest.mark.parametrize("n,t", [(1, 1), (2, 7), (3, 64), (5, 33), (8, 64)])
def test_bruteforce_python_complex(oracle_mod, n, t):
    # Eq. 1 through Python's own complex multiply and conjugate
    x, qr, qi = parts(2, t, n, seed=100 + n * 7 + t)
    got = oracle_mod.correlate(x)
    for ch in range(2):
        k = 0
        for i in range(n):
            for j in range(i, n):
                v = 0j
                for s in range(t):
                    xi = complex(int(qr[ch, s, i]), int(qi[ch, s, i]))
                    xj = complex(int(qr[ch, s, j]), int(qi[ch, s, j]))
                    v += xi * xj.conjugate()
                assert got[ch, k, 0] == int(v.real) and got[ch, k, 1] == int(v.imag), (ch, i, j)
                k += 1


@pytest.mark.parametrize("f,t,n,common", [(3, 300, 37, 0.0), (2, 1000, 64, 0.3), (1, 129, 100, 0.0)])
def test_numpy_complex_matmul(oracle_mod, f, t, n, common):
    # V = X^T conj(X) with numpy's complex128 matmul (exact: sums << 2^53)
    x, qr, qi = parts(f, t, n, seed=7 + n, common=common)
    z = qr.astype(np.float64) + 1j * qi.astype(np.float64)
    ref = np.matmul(np.transpose(z, (0, 2, 1)), np.conj(z))
    i, j = np.triu_indices(n)
    got = oracle_mod.correlate(x)
    assert np.array_equal(got[..., 0], ref[:, i, j].real.astype(np.int64))
    assert np.array_equal(got[..., 1], ref[:, i, j].imag.astype(np.int64))


def test_exhaustive_byte_pairs(oracle_mod):
    # every (x0, x1) pair of 4-bit complex values, one channel per pair, T = 1
    vals = np.arange(-8, 8)
    re0, im0, re1, im1 = np.meshgrid(vals, vals, vals, vals, indexing="ij")
    re0, im0, re1, im1 = (a.reshape(-1) for a in (re0, im0, re1, im1))
    x = np.stack([synth.pack(re0, im0), synth.pack(re1, im1)], axis=1).reshape(-1, 1, 2)
    got = oracle_mod.correlate(x)
    z0 = re0 + 1j * im0
    z1 = re1 + 1j * im1
    for k, ref in enumerate((z0 * np.conj(z0), z0 * np.conj(z1), z1 * np.conj(z1))):
        assert np.array_equal(got[:, k, 0], ref.real.astype(np.int64))
        assert np.array_equal(got[:, k, 1], ref.imag.astype(np.int64))


def test_offset_route_matches(oracle_mod):
    # the paper's Eq. 3 route (unsigned products + running-sum offsets)
    for (f, t, n, seed) in [(2, 256, 16, 1), (1, 333, 31, 2), (3, 64, 7, 3)]:
        x = synth.uniform_bytes(f, t, n, seed).numpy()
        assert np.array_equal(oracle_mod.offset_route(x), oracle_mod.correlate(x))


def test_hermitian_and_upper_consistency(oracle_mod):
    x = synth.uniform_bytes(2, 200, 19, 11).numpy()
    full = oracle_mod.full_matrix(x)
    assert np.array_equal(full[..., 0], np.transpose(full[..., 0], (0, 2, 1)))
    assert np.array_equal(full[..., 1], -np.transpose(full[..., 1], (0, 2, 1)))
    assert np.array_equal(upper(full), oracle_mod.correlate(x))


def test_autocorrelations(oracle_mod):
    x, qr, qi = parts(2, 500, 24, seed=5)
    vis = oracle_mod.correlate(x)
    n = 24
    diag = [i * (2 * n - i + 1) // 2 for i in range(n)]
    power = (qr * qr + qi * qi).sum(axis=1)          # [F][N]
    assert np.array_equal(vis[:, diag, 1], np.zeros_like(power))
    assert np.array_equal(vis[:, diag, 0], power)
    assert (vis[:, diag, 0] >= 0).all()


@pytest.mark.parametrize("a,b", [(-8, -8), (7, 7), (-8, 7), (3, -5), (0, 0), (1, 0)])
def test_constant_input_closed_form(oracle_mod, a, b):
    t, n = 97, 9
    x = np.full((1, t, n), synth.pack(a, b), dtype=np.uint8)
    vis = oracle_mod.correlate(x)
    assert (vis[..., 0] == t * (a * a + b * b)).all()
    assert (vis[..., 1] == 0).all()


def test_all_zero_bytes_is_128T(oracle_mod):
    # byte 0x00 encodes (-8, -8): |x|^2 = 128 per sample
    t, n = 1000, 5
    vis = oracle_mod.correlate(np.zeros((1, t, n), dtype=np.uint8))
    assert (vis[..., 0] == 128 * t).all() and (vis[..., 1] == 0).all()


def test_per_element_constants(oracle_mod):
    # x_i constant in time: V_ij = T * x_i * conj(x_j)
    rng = np.random.default_rng(3)
    n, t = 12, 50
    re = rng.integers(-8, 8, size=n)
    im = rng.integers(-8, 8, size=n)
    x = np.broadcast_to(synth.pack(re, im), (1, t, n)).copy()
    vis = oracle_mod.correlate(x)
    z = re + 1j * im
    i, j = np.triu_indices(n)
    ref = t * z[i] * np.conj(z[j])
    assert np.array_equal(vis[0, :, 0], ref.real.astype(np.int64))
    assert np.array_equal(vis[0, :, 1], ref.imag.astype(np.int64))


def test_time_additivity_and_accumulate(oracle_mod):
    x = synth.uniform_bytes(2, 300, 13, 21).numpy()
    whole = oracle_mod.correlate(x)
    first = oracle_mod.correlate(x[:, :117])
    both = oracle_mod.correlate(x[:, 117:], prev=first)
    assert np.array_equal(whole, both)


def test_element_permutation_covariance(oracle_mod):
    x = synth.uniform_bytes(1, 80, 11, 8).numpy()
    perm = np.random.default_rng(0).permutation(11)
    full = oracle_mod.full_matrix(x)
    fullp = oracle_mod.full_matrix(x[:, :, perm])
    assert np.array_equal(fullp, full[:, perm][:, :, perm])


def test_entries_match_full(oracle_mod):
    x = synth.uniform_bytes(3, 100, 20, 4).numpy()
    vis = oracle_mod.correlate(x)
    pairs = oracle_mod.tri_pairs(20)
    rng = np.random.default_rng(1)
    pick = rng.integers(0, len(pairs), size=50)
    chans = rng.integers(0, 3, size=50)
    fij = np.stack([chans, pairs[pick, 0], pairs[pick, 1]], axis=1)
    got = oracle_mod.entries(x, fij)
    assert np.array_equal(got, vis[chans, pick])


def test_empty_time_axis(oracle_mod):
    vis = oracle_mod.correlate(np.zeros((2, 0, 4), dtype=np.uint8))
    assert (vis == 0).all()


def test_int32_boundary(oracle_mod):
    # T = 16 777 215 samples of (-8,-8): Re = 128*T = 2 147 483 520 fits int32;
    # one more sample would not
    from paper_1503_06203_amd import metrics
    t = metrics.MAX_SAMPLES
    vis = oracle_mod.correlate(np.zeros((1, t, 1), dtype=np.uint8))
    assert vis[0, 0, 0] == 128 * t == 2_147_483_520
    assert oracle_mod.to_int32(vis)[0, 0, 0] == 2_147_483_520
    with pytest.raises(OverflowError):
        oracle_mod.to_int32(vis + 128)


def test_paper_numbers():
    from paper_1503_06203_amd import metrics
    g = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    assert metrics.OPS_PER_CMAC == g["ops_per_cmac"]["value"]
    p = g["r9_280x_peak"]
    peak = p["clock_hz"] * p["compute_units"] * p["cores_per_cu"] * p["ops_per_mad"]
    assert round(peak / 1e12, 1) == p["quoted_tops"]
    n = g["n2048_unpacked_matrices_per_s"]["n"]
    per_matrix = metrics.effective_ops(n, 1, 1)          # Eq. 2
    assert per_matrix == 16_785_408
    assert round(peak / per_matrix / 1e3) == g["n2048_unpacked_matrices_per_s"]["quoted_thousands"]
    packed = g["n2048_packed_matrices_per_s"]["quoted"]
    assert round(packed * per_matrix / 1e12, 1) == g["packed_effective_tops"]["quoted"]
    assert round(100 * packed / (peak / per_matrix)) == g["packed_vs_unpacked_percent"]["quoted"]
    fig = g["fig1_tiling"]
    assert metrics.tile_count(fig["n"], fig["tile"]) == fig["tiles"]
    acc = g["packed_16bit_accumulation"]
    assert 15 * 15 == acc["max_product"]              # encoded fields lie in [0, 15]
    assert acc["container_max"] // acc["max_product"] == acc["steps"]


# ---- gated correlation (sum per gate bin) -------------------------------------------

def test_gated_bruteforce(oracle_mod):
    # tiny case through Python complex arithmetic: gate of each sample by block
    n, t, block = 3, 11, 3
    x, qr, qi = parts(1, t, n, seed=404)
    gate_of_block = [1, 0, 0xFF, 1]            # samples 0-2 -> 1, 3-5 -> 0, 6-8 dropped, 9-10 -> 1
    got = oracle_mod.correlate_gated(x, gate_of_block, block, 2)
    gate_of_sample = [gate_of_block[s // block] for s in range(t)]
    for g in range(2):
        k = 0
        for i in range(n):
            for j in range(i, n):
                v = 0j
                for s in range(t):
                    if gate_of_sample[s] != g:
                        continue
                    xi = complex(int(qr[0, s, i]), int(qi[0, s, i]))
                    xj = complex(int(qr[0, s, j]), int(qi[0, s, j]))
                    v += xi * xj.conjugate()
                assert got[g, 0, k, 0] == int(v.real) and got[g, 0, k, 1] == int(v.imag), (g, i, j)
                k += 1


def test_gated_invariants(oracle_mod):
    x = synth.uniform_bytes(2, 1000, 24, seed=405).numpy()
    plain = oracle_mod.correlate(x)
    nb = (1000 + 63) // 64
    # one gate holding every block is the plain correlation
    one = oracle_mod.correlate_gated(x, [0] * nb, 64, 1)
    assert np.array_equal(one[0], plain)
    # gates partition the samples: their sum is the plain correlation
    rng = np.random.default_rng(3)
    sched = rng.integers(0, 3, nb)
    three = oracle_mod.correlate_gated(x, sched, 64, 3)
    assert np.array_equal(three.sum(axis=0), plain)
    # a dropped block is simply absent; an unused gate is zero
    sched2 = sched.copy()
    sched2[5] = 0xFF
    dropped = oracle_mod.correlate_gated(x, sched2, 64, 4)
    block5 = oracle_mod.correlate(np.ascontiguousarray(x[:, 320:384]))
    assert np.array_equal(dropped[:3].sum(axis=0) + block5, plain)
    assert not dropped[3].any()


# ---- delay compensation ---------------------------------------------------------------

def test_delayed_bruteforce(oracle_mod):
    n, t = 3, 9
    delays = [2, 0, 1]
    d = max(delays)
    x, qr, qi = parts(1, t + d, n, seed=406)
    got = oracle_mod.correlate_delayed(x, delays)
    k = 0
    for i in range(n):
        for j in range(i, n):
            v = 0j
            for s in range(t):
                si, sj = d + s - delays[i], d + s - delays[j]
                xi = complex(int(qr[0, si, i]), int(qi[0, si, i]))
                xj = complex(int(qr[0, sj, j]), int(qi[0, sj, j]))
                v += xi * xj.conjugate()
            assert got[0, k, 0] == int(v.real) and got[0, k, 1] == int(v.imag), (i, j)
            k += 1


def test_delayed_special_cases(oracle_mod):
    x = synth.uniform_bytes(2, 300, 16, seed=407).numpy()
    # no delays: the last T samples, correlated plainly
    zero = oracle_mod.correlate_delayed(x[:, :, :], [0] * 16)
    assert np.array_equal(zero, oracle_mod.correlate(x))
    # one common delay c with max delay D = c: the first T samples
    common = oracle_mod.correlate_delayed(x, [44] * 16)
    assert np.array_equal(common, oracle_mod.correlate(np.ascontiguousarray(x[:, :256])))
