"""Host-side check of the index algebra behind the lane-shared shell reads of the
collide kernels (lane_x, GlobalShell::elem_share, diag_plane16, lane_xp1 and
k_att_x in hslb_kernels.hip), with the rotation amounts transcribed here.

A lane holds node (x, b0) of a periodic x-row of nx nodes (b is the second axis
of the face-diagonal plane: y for the xy plane, z for the xz plane); "the value
lane x + k loaded" is a rotation by k.  For every sigma 2..8, every corner
(l + ka, +-(l + kb)) of the two face-diagonal points (1, 1) and (1, -1), and
every lane of rows of 16, 64, 128 and 256 nodes, the node a shared read comes
from must be the node the element needs:
  - (n, j) at r + d and r - d;
  - the contact value G+ at the midpoint of (r, r + d), stored at the lower
    node r + floor(d / 2) in the sub-lattice of the parities of d, and G- at
    r + floor(-d / 2) in the same sub-lattice.
"""
import pytest


def ell(s):
    l = 0
    while 2 * (l + 1) ** 2 <= s * s:
        l += 1
    return l


def fd2(d):
    return (d - (d & 1)) // 2


def slot(da, db):
    return (da & 1, db & 1)


class Row:
    """A row of nx lanes: lane x holds node x; loads are functions of the node."""

    def __init__(self, nx):
        self.nx = nx

    def rot(self, loaded, k):
        """The values of `loaded` (indexed by lane) held by lane x + k."""
        return [loaded[(x + k) % self.nx] for x in range(self.nx)]


def nj_at(x, b):
    return ("nj", x, b)


def g_at(x, b, s):
    return ("G", x, b, s)


def needed(nx, x, b0, LA, DB):
    """(qp, qm, gp, gm) an element with corner d = (LA, DB) needs at lane x."""
    return (nj_at((x + LA) % nx, b0 + DB), nj_at((x - LA) % nx, b0 - DB),
            g_at((x + fd2(LA)) % nx, b0 + fd2(DB), slot(LA, DB)),
            g_at((x + fd2(-LA)) % nx, b0 + fd2(-DB), slot(LA, DB)))


@pytest.mark.parametrize("nx", [16, 64, 128, 256])
@pytest.mark.parametrize("sigma", range(2, 9))
def test_x_neighbour_corner_reads(nx, sigma):
    """elem_share (ROT 1/2/3): the corner (l + 1, DB) takes its (n, j) from the
    lane of x + 1 (r + d) and of x - 1 (r - d) of the corner (l, DB); its own
    contact values are loaded."""
    LL, b0, row = ell(sigma), 0, Row(nx)
    for DB in (LL, LL + 1, -LL, -(LL + 1)):
        qp0 = [nj_at((x + LL) % nx, b0 + DB) for x in range(nx)]
        qm0 = [nj_at((x - LL) % nx, b0 - DB) for x in range(nx)]
        qp1, qm1 = row.rot(qp0, +1), row.rot(qm0, -1)
        for x in range(nx):
            want = needed(nx, x, b0, LL + 1, DB)
            assert (qp1[x], qm1[x]) == want[:2], (sigma, nx, DB, x)


@pytest.mark.parametrize("sigma", range(2, 9))
def test_mirrored_points_on_16_node_rows(sigma):
    """diag_plane16 (ROT 2): per offset LB one (n, j) load P at r + (l, LB) and
    one M at r - (l, LB); corner (LA, LB) of the point (1, 1) reads P and M
    rotated by LA - l and -(LA - l); corner (LA, -LB) of the point (1, -1)
    reads M rotated by l + LA and P by -(l + LA), and its G+ / G- are the
    point (1, 1) corner's G- / G+ rotated by +LA / -LA."""
    nx, LL, b0, row = 16, ell(sigma), 0, Row(16)
    assert 2 * LL + 1 < 16
    for kb in (0, 1):
        LB = LL + kb
        P = [nj_at((x + LL) % nx, b0 + LB) for x in range(nx)]
        M = [nj_at((x - LL) % nx, b0 - LB) for x in range(nx)]
        for ka in (0, 1):
            LA = LL + ka
            gp = [g_at((x + fd2(LA)) % nx, b0 + fd2(LB), slot(LA, LB)) for x in range(nx)]
            gm = [g_at((x + fd2(-LA)) % nx, b0 + fd2(-LB), slot(LA, LB)) for x in range(nx)]
            q = (row.rot(P, ka), row.rot(M, -ka), gp, gm)
            r = (row.rot(M, LL + LA), row.rot(P, -(LL + LA)), row.rot(gm, LA), row.rot(gp, -LA))
            for x in range(nx):
                assert tuple(v[x] for v in q) == needed(nx, x, b0, LA, LB), (sigma, ka, kb, x)
                assert tuple(v[x] for v in r) == needed(nx, x, b0, LA, -LB), (sigma, ka, kb, x)


@pytest.mark.parametrize("nx,waves", [(128, 2), (256, 4)])
@pytest.mark.parametrize("sigma", range(2, 9))
def test_row_edge_exchange_over_waves(nx, waves, sigma):
    """ROT 3: a wave rotation inside each 64-lane wave gives every lane but the
    row-edge ones its x + 1 (x - 1) neighbour's value; lane 63 (lane 0) takes
    the entry lane 0 (lane 63) of the next (previous) wave of the same row,
    periodic over the row, stored in s_xedge."""
    LL, b0 = ell(sigma), 0
    for DB in (LL, LL + 1, -LL, -(LL + 1)):
        qp0 = [nj_at((x + LL) % nx, b0 + DB) for x in range(nx)]
        qm0 = [nj_at((x - LL) % nx, b0 - DB) for x in range(nx)]
        edge_p = [qp0[64 * w] for w in range(waves)]        # lane 0 of each wave, r + d
        edge_m = [qm0[64 * w + 63] for w in range(waves)]   # lane 63 of each wave, r - d
        for x in range(nx):
            w, lane = divmod(x, 64)
            rp = qp0[64 * w + (lane + 1) % 64]              # wave_rol:1
            rm = qm0[64 * w + (lane - 1) % 64]              # wave_ror:1
            wn, wp = (w + 1) % waves, (w - 1) % waves
            if lane == 63:
                rp = edge_p[wn]
            if lane == 0:
                rm = edge_m[wp]
            assert (rp, rm) == needed(nx, x, b0, LL + 1, DB)[:2], (sigma, nx, DB, x)


@pytest.mark.parametrize("nx", [16, 64])
def test_x_plus_one_and_attraction_taps(nx):
    """lane_xp1: the contact-value kernel's eta_bar at x + 1 and the attraction
    x-pass's taps n(x + m - R), m = 0..2R (R up to 30, more than a row), from
    one load of n(x - R) rotated m times by one lane."""
    row = Row(nx)
    eb = list(range(nx))
    assert row.rot(eb, 1) == [(x + 1) % nx for x in range(nx)]
    for R in (0, 4, 12, 30):
        v = [(x - R) % nx for x in range(nx)]
        for m in range(2 * R + 1):
            assert v == [(x + m - R) % nx for x in range(nx)], (R, m)
            v = row.rot(v, 1)
