"""Host replay of the halo ring of the brick weight gradient (no GPU).

k_wgrad_tr walks each block's bricks in z order within an (x, y) column and
keeps the input halo in 8 plane slots (input plane z in slot z mod 8, 256
items each): a brick after its z neighbour copies only its 4 new planes.
This test transcribes the kernel's copy and read index arithmetic and
replays the copies of whole brick ranges into a model of LDS.  Every
transposing read of every wave, step and tap (a subset of lanes) must see
the element the plain layout (the brick's 6 halo planes side by side, 240
items each) holds at the matching address, at the same offset within its
16-byte item, and every copy must land inside the ring or the
output-gradient region.  The kernel itself is held against the oracle by
tests/test_gpu_nn.py."""
import pytest

ROW = 20                  # voxel slots per halo row (18 + 2 padding)
PLANE_ITEMS = 256         # 16-byte items per ring slot (6 rows of 40, then padding)
RING = 8
HALO_ITEMS = RING * PLANE_ITEMS
PLAIN_HALO_BUF = 1472     # the plain layout's halo region, whole copies of 64 items


def replay(G, per, RS, n=2, lane_step=3):
    nbx, nby, nbz = G >> 4, G >> 2, G >> 2
    nbricks = n * nbz * nby * nbx
    dy_row = 40 if RS == 1 else 66
    dy_items = 16 * dy_row
    dy_buf = (dy_items + 63) // 64 * 64

    def brick(b):
        z0 = (b % nbz) * 4
        b //= nbz
        x0 = (b % nbx) * 16
        b //= nbx
        return x0, (b % nby) * 4, z0, b // nby

    def halo(smp, xx, yy, zz, half, ok):
        if not ok or not (0 <= xx < G and 0 <= yy < G and 0 <= zz < G):
            return 0
        return ("x", smp, zz, yy, xx, half)

    def dy(smp, x0, y0, z0, t):
        row, it = divmod(t, dy_row)
        px, c8 = divmod(it, 2 * RS)
        if t >= dy_items or px >= 16:
            return 0
        return ("d", smp, z0 + ((row >> 2) & 3), y0 + (row & 3), x0 + (px & 15), c8)

    reads = 0
    for b0 in range(0, nbricks, per):
        b1 = min(b0 + per, nbricks)
        lds = {}
        for b in range(b0, b1):
            x0, y0, z0, smp = brick(b)
            fresh = b == b0 or z0 == 0
            zfirst = z0 - 1 if fresh else z0 + 1
            nh = (6 if fresh else 4) * (PLANE_ITEMS // 64)
            for j in range(nh + dy_buf // 64):
                for ln in range(64):
                    if j < nh:
                        zz = zfirst + (j >> 2)
                        t = (j & 3) * 64 + ln
                        half, hv = t & 1, t >> 1
                        hx, hy = hv % ROW, hv // ROW
                        dst = (zz & (RING - 1)) * PLANE_ITEMS + (j & 3) * 64 + ln
                        assert 0 <= dst < HALO_ITEMS
                        lds[dst] = halo(smp, x0 + hx - 1, y0 + hy - 1, zz, half, hy < 6 and hx < 18)
                    else:
                        dst = HALO_ITEMS + (j - nh) * 64 + ln
                        assert dst < HALO_ITEMS + dy_buf
                        lds[dst] = dy(smp, x0, y0, z0, (j - nh) * 64 + ln)

            def plain(t):  # the plain layout's item t for this brick
                if t >= PLAIN_HALO_BUF:
                    return dy(smp, x0, y0, z0, t - PLAIN_HALO_BUF)
                half, hv = t & 1, t >> 1
                hx, hy, hz = hv % ROW, (hv // ROW) % 6, hv // (6 * ROW)
                return halo(smp, x0 + hx - 1, y0 + hy - 1, z0 + hz - 1, half, t < 1440 and hx < 18)

            for wave in range(9):
                dzw, dyw = wave // 3, wave % 3
                for lane in range(0, 64, lane_step):
                    r, q = lane & 15, lane >> 4
                    e, ac = r >> 2, r & 3
                    a_rel = ((q & 1) * dy_row + (8 * (q >> 1) + e) * 2 * RS) * 16 + ac * 8
                    b_plain = (((q & 1) + dyw) * ROW + dzw * 6 * ROW + 8 * (q >> 1) + e) * 32 + ac * 8
                    b_ring = (((q & 1) + dyw) * ROW + 8 * (q >> 1) + e) * 32 + ac * 8
                    bp = [b_ring + ((z0 - 1 + dzw + p) & (RING - 1)) * PLANE_ITEMS * 16 for p in range(4)]
                    for s in range(8):
                        ra = ((s >> 1) * 4 + 2 * (s & 1)) * dy_row * 16
                        pairs = []
                        for m in range(RS):
                            for k in (m * 32, 4 * 32 * RS + m * 32):
                                pairs.append((PLAIN_HALO_BUF * 16 + a_rel + ra + k,
                                              HALO_ITEMS * 16 + a_rel + ra + k))
                        for dx in range(3):
                            for k in (0, 4):
                                pairs.append((b_plain + (((s >> 1) * 6 + 2 * (s & 1)) * ROW + dx + k) * 32,
                                              bp[s >> 1] + (2 * (s & 1) * ROW + dx + k) * 32))
                        for ap, ar in pairs:
                            assert ap % 16 == ar % 16
                            assert plain(ap // 16) == lds.get(ar // 16, "unwritten"), (b, wave, lane, s)
                            reads += 1
    return reads


@pytest.mark.parametrize("G,per,RS", [(16, 1, 1), (16, 3, 1), (16, 5, 2), (32, 7, 1), (32, 20, 2)])
def test_ring_reads_match_the_plain_halo(G, per, RS):
    assert replay(G, per, RS, n=1 if G == 32 else 2, lane_step=3 if G == 16 else 7) > 0
