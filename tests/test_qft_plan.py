"""Host checks of the FFT block passes of sv_qft (no GPU): the planner's
index maps are bijections within bounds, and a numpy replay of the passes
with exactly the kernel's data movement (tiles, stage register/thread maps,
decimation-in-frequency order, twiddles) equals the DFT that defines the QFT
(sec. 2.3.2), with the range left bit-reversed as the circuit leaves it
before its swaps."""

import ctypes

import numpy as np
import pytest

W = 42


def plan(n, q0, m):
    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    cnt = ctypes.c_int64()
    assert L.sv_qft_plan(n, q0, m, None, 0, ctypes.byref(cnt)) == 0
    out = np.zeros(max(1, cnt.value) * W, dtype=np.int32)
    assert L.sv_qft_plan(n, q0, m, out.ctypes.data_as(ctypes.c_void_p), cnt.value, ctypes.byref(cnt)) == 0
    return [out[p * W:(p + 1) * W] for p in range(cnt.value)]


def dep(x, pos):
    e = 0
    for i, p in enumerate(pos):
        e |= ((x >> i) & 1) << int(p)
    return e


def rev(x, nb):
    return int(format(x, "0%db" % nb)[::-1], 2) if nb else 0


def stage_indices(regb, thrb):
    """e index of (thread, register) for a stage map."""
    idx = np.zeros((256, 16), dtype=np.int64)
    for t in range(256):
        to = dep(t, thrb)
        for r in range(16):
            idx[t, r] = to | dep(r, regb)
    return idx


def dif(v, D, sign):
    """The kernel's radix-2 DIF over the high D register bits of v[..., 16]."""
    v = v.copy()
    BB = 4 - D
    for lsp in range(D - 1, -1, -1):
        sp = 1 << lsp
        for i in range(1 << D):
            if i & sp:
                continue
            j = i & (sp - 1)
            w = np.exp(2j * np.pi * sign * j / (2 * sp))
            for b in range(1 << BB):
                r0, r1 = (i << BB) | b, ((i + sp) << BB) | b
                x, y = v[..., r0].copy(), v[..., r1].copy()
                v[..., r0] = x + y
                v[..., r1] = (x - y) * w
    return v


def replay(a, n, q0, m, sign):
    a = a.astype(np.complex128).copy()
    for P in plan(n, q0, m):
        blo, t, A, B, lo, eb = (int(x) for x in P[:6])
        ebits = [int(x) for x in P[6:18]]
        if t == 12:
            # the 12-bit block on bits [0, 12): its kernel's three-level DIF
            # leaves w at rev_12(w); no lower qubits, scale 2^-6
            assert blo == 0 and lo == 0 and ebits == list(range(12)) and all(int(x) == -1 for x in P[18:42])
            A3 = a.reshape(-1, 4096)
            F = np.fft.ifft(A3, axis=1, norm="ortho") if sign > 0 else np.fft.fft(A3, axis=1, norm="ortho")
            r = np.array([rev(w, 12) for w in range(4096)])
            out = np.empty_like(F)
            out[:, r] = F
            a = out.reshape(-1)
            continue
        s1r, s1t = P[18:22], P[22:30]
        s2r, s2t = P[30:34], P[34:42]
        assert len(set(ebits)) == 12 and all(0 <= b < n for b in ebits) and ebits == sorted(ebits)
        assert ebits[eb] == blo and ebits[eb:eb + t] == list(range(blo, blo + t))
        i1 = stage_indices(s1r, s1t)
        assert sorted(i1.ravel()) == list(range(4096))
        assert all(int(x) == eb + B + k for k, x in enumerate(s1r[4 - A:]))
        if B:
            i2 = stage_indices(s2r, s2t)
            assert sorted(i2.ravel()) == list(range(4096))
            assert all(int(x) == eb + k for k, x in enumerate(s2r[4 - B:]))
        goff = np.array([dep(e, ebits) for e in range(4096)], dtype=np.int64)
        others = [b for b in range(n) if b not in ebits]
        btw = blo + t - lo
        scale = 2.0 ** (-t / 2)
        seen = np.zeros(1 << n, dtype=bool)
        for tile in range(1 << (n - 12)):
            base = dep(tile, others)
            g = base | goff
            assert not seen[g].any()
            seen[g] = True
            x = a[g]                                 # LDS tile, by e
            v = x[i1]                                # stage 1 registers
            v = dif(v, A, sign)
            if B:
                v0 = (i1[:, 0] >> eb) & ((1 << B) - 1)   # fixed per thread when A = 4
                assert A == 4 and np.all(((i1 >> eb) & ((1 << B) - 1)) == v0[:, None])
                z0 = np.exp(2j * np.pi * sign * v0 / (1 << t))
                for w0 in range(1, 16):
                    v[:, rev(w0, 4)] *= z0 ** w0
            x[i1] = v
            if B:
                v = dif(x[i2], B, sign)
                x[i2] = v
            e = np.arange(4096)
            d1 = (e >> (eb + B)) & ((1 << A) - 1)
            d0 = (e >> eb) & ((1 << B) - 1)
            w = np.array([rev(int(p), A) for p in d1]) | (np.array([rev(int(q), B) for q in d0]) << A)
            Lv = (g >> lo) & ((1 << (blo - lo)) - 1)
            k = (w * Lv) & ((1 << btw) - 1)
            a[g] = x * np.exp(2j * np.pi * sign * k / (1 << btw)) * scale
        assert seen.all()
    return a


def reference(a, n, q0, m, sign):
    """DFT over qubits q0..q0+m-1 (index bits [lo, lo+m)) then the range's
    bits reversed."""
    lo = n - q0 - m
    A = a.reshape(1 << q0, 1 << m, 1 << lo)
    F = np.fft.ifft(A, axis=1, norm="ortho") if sign > 0 else np.fft.fft(A, axis=1, norm="ortho")
    r = np.array([rev(y, m) for y in range(1 << m)])
    out = np.empty_like(F)
    out[:, r, :] = F
    return out.reshape(-1)


@pytest.mark.parametrize("n,q0,m", [(12, 0, 12), (13, 0, 13), (14, 0, 14), (14, 2, 9), (13, 5, 3), (14, 0, 5),
                                    (12, 11, 1), (14, 3, 11), (13, 1, 6), (14, 6, 8), (14, 1, 13), (13, 1, 12),
                                    (16, 0, 16), (14, 2, 12), (19, 0, 19), (15, 1, 13)])
@pytest.mark.parametrize("sign", [1, -1])
def test_replay_equals_dft(n, q0, m, sign):
    rng = np.random.default_rng(n * 100 + q0 * 10 + m)
    a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    got = replay(a, n, q0, m, sign)
    want = reference(a, n, q0, m, sign)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want)) * 100


def test_plan_blocks_cover_range():
    for n in (12, 20, 30, 36):
        for q0, m in ((0, n), (1, n - 1), (3, 7), (n - 1, 1)):
            ps = plan(n, q0, m)
            lo = n - q0 - m
            blocks = sorted((int(P[0]), int(P[1])) for P in ps)
            pos = lo
            for blo, t in blocks:
                assert blo == pos and (1 <= t <= 8 or (t == 12 and blo == 0 == lo))
                pos += t
            assert pos == lo + m
    from paper_quant_ph_0201042_amd import _lib

    L = _lib.load()
    cnt = ctypes.c_int64()
    assert L.sv_qft_plan(11, 0, 11, None, 0, ctypes.byref(cnt)) == -1
    assert L.sv_qft_plan(14, 3, 12, None, 0, ctypes.byref(cnt)) == -1


def test_twelve_bit_kernel_maps():
    # the fixed maps of the 12-bit block kernel: every stage visits each tile
    # index once, and the DFT bits are the register bits
    tid = np.arange(256)[:, None]
    r = np.arange(16)[None, :]
    s1 = (r << 8) | tid
    e2 = ((tid >> 4) << 8) | (tid & 15)
    s2 = e2 | (r << 4)
    s3 = (tid << 4) | r
    for idx in (s1, s2, s3):
        assert sorted(idx.ravel()) == list(range(4096))
    assert np.all((s1 >> 8) == r) and np.all(((s2 >> 4) & 15) == r) and np.all((s3 & 15) == r)


def test_twelve_bit_dif_order():
    # DFT_16 over bits 8..11, twiddle e^{2 pi i s v_low w0 / 4096}, DFT_16
    # over bits 4..7, twiddle e^{2 pi i s v_lo w1 / 256}, DFT_16 over bits
    # 0..3 (each DIF, output at bit-reversed register positions) equals the
    # 4096-point DFT written at rev_12(w)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(4096) + 1j * rng.standard_normal(4096)
    for sign in (1, -1):
        t = x.copy()
        tid = np.arange(256)
        v = t[(np.arange(16)[None, :] << 8) | tid[:, None]]          # [tid, r]
        v = dif(v, 4, sign)
        z1 = np.exp(2j * np.pi * sign * tid / 4096)
        for w in range(1, 16):
            v[:, rev(w, 4)] *= z1 ** w
        t[(np.arange(16)[None, :] << 8) | tid[:, None]] = v
        e2 = ((tid >> 4) << 8) | (tid & 15)
        idx = e2[:, None] | (np.arange(16)[None, :] << 4)
        v = dif(t[idx], 4, sign)
        z2 = np.exp(2j * np.pi * sign * (tid & 15) / 256)
        for w in range(1, 16):
            v[:, rev(w, 4)] *= z2 ** w
        t[idx] = v
        idx = (tid[:, None] << 4) | np.arange(16)[None, :]
        t[idx] = dif(t[idx], 4, sign)
        F = np.fft.ifft(x, norm="forward") if sign > 0 else np.fft.fft(x)
        want = np.empty_like(F)
        want[[rev(w, 12) for w in range(4096)]] = F
        assert np.max(np.abs(t - want)) < 1e-9



def test_plan_balanced_block_sizes():
    # as few blocks of at most 8 bits as the range above the 12-bit block
    # needs, of balanced sizes (longer contiguous runs in each tile)
    def sizes(n, q0, m):
        return [int(P[1]) for P in plan(n, q0, m)]

    assert sizes(28, 0, 28) == [8, 8, 12]
    assert sizes(29, 0, 29) == [6, 6, 5, 12]
    assert sizes(30, 0, 30) == [6, 6, 6, 12]
    assert sizes(33, 0, 33) == [7, 7, 7, 12]
    assert sizes(22, 2, 18) == [6, 6, 6]
    assert sizes(20, 3, 9) == [5, 4]
    for n in range(12, 37):
        for q0, m in ((0, n), (1, n - 1), (n - 9, 9)):
            s = sizes(n, q0, m)
            last = 12 if n - q0 - m == 0 and m >= 12 else 0
            upper = s[:-1] if last else s
            assert not last or s[-1] == 12
            assert len(upper) == -(-(m - last) // 8)
            assert max(upper, default=0) - min(upper, default=0) <= 1
