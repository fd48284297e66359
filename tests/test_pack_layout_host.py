"""Host replay of the weight packing's tiles (no GPU).

k_pack_all writes each layer's transposed, tap-flipped BF16 copy
wt[cinp][kpad_t] (k = tap * ys + co) in LDS tiles of 16 input channels x 64
k entries: 4 lanes per k entry read 4 input channels each from the master
weights w[co][tap][ci], then 16 lanes per channel write 4 consecutive k
entries.  This test transcribes that tile arithmetic and replays it for
many layer shapes: every element of the padded array, zero padding
included, must be written exactly once and equal the per-element
definition (the padding matters because a stale value there would only
show on reused memory).  The packed values themselves are held against the
oracle by the network tests on the GPU."""
import itertools

import numpy as np


def ru(a, m):
    return (a + m - 1) // m * m


def element(L, idx, w):
    """wt element idx by its definition: w[co][taps - 1 - t][real channel]."""
    ci, k = divmod(idx, L["kpad_t"])
    if ci >= L["cin"] or k >= L["taps"] * L["ys"]:
        return 0.0
    t, co = divmod(k, L["ys"])
    if co >= L["cout"] or not (ci >= L["c1s"] or ci < L["c1"]):
        return 0.0
    cir = ci if ci < L["c1s"] else L["c1"] + (ci - L["c1s"])
    return w[(co * L["taps"] + (L["taps"] - 1 - t)) * L["cin_real"] + cir]


def test_transposed_tiles_cover_the_padded_array_once():
    rng = np.random.default_rng(0)
    shapes = 0
    for c1, c2, cout, taps in itertools.product([4, 16, 24], [0, 16, 32], [4, 16, 48], [1, 27]):
        c1s = ru(c1, 8)
        cin = c1s + c2
        ys = ru(cout, 8)
        L = dict(cin=cin, c1=c1, c1s=c1s, cout=cout, taps=taps, ys=ys, cin_real=c1 + c2,
                 kpad_t=ru(taps * ys, 32), cinp=ru(cin, 16))
        kpad_t, cinp = L["kpad_t"], L["cinp"]
        assert cinp % 16 == 0 and kpad_t % 4 == 0   # what the host checks before the launch
        w = rng.standard_normal(cout * taps * (c1 + c2))
        out = np.full(cinp * kpad_t, np.nan)
        writes = np.zeros(cinp * kpad_t, int)
        nkt = (kpad_t + 63) // 64
        for b in range((cinp // 16) * nkt):
            ci0, k0 = (b // nkt) * 16, (b % nkt) * 64
            tile = np.zeros((64, 17))
            for tid in range(256):
                kk, c4 = tid >> 2, (tid & 3) * 4
                for u in range(4):
                    idx = (ci0 + c4 + u) * kpad_t + k0 + kk
                    tile[kk, c4 + u] = element(L, idx, w) if k0 + kk < kpad_t else 0.0
            for tid in range(256):
                cl, k4 = tid >> 4, (tid & 15) * 4
                if k0 + k4 >= kpad_t:
                    continue
                for u in range(4):
                    i = (ci0 + cl) * kpad_t + k0 + k4 + u
                    out[i] = tile[k4 + u, cl]
                    writes[i] += 1
        ref = np.array([element(L, i, w) for i in range(cinp * kpad_t)])
        assert (writes == 1).all(), L
        assert np.array_equal(out, ref), L
        shapes += 1
    assert shapes == 54
