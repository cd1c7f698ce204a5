"""Host-side bounds check of the LDS-staged collide kernel's index arithmetic
(k_collide_tiles: copy_tile and StagedShell in hslb_kernels.hip), with its
formulas transcribed here: the global-to-LDS placement (the wave issuing
entries [256 k + 64 w, +64) writes them to the region base + that range), every
LDS entry inside the block's array, every staged read returning exactly the
element the direct kernel's load_pair reads for the same pair, and every global
read inside its field (x, y wrapped once, padded z inside the halo layers).
Tiles at the lattice's corners and edges, the lowest and highest fluid layer,
sigma 2..8."""
import pytest

TX, TY, GH = 64, 4, 4
STAGE_BG = False  # the kernel stages phase B's contact values only with STAGE_BG
GWX = TX + 2 * GH
def ell(s):
    l = 0
    while 2 * (l + 1) ** 2 <= s * s: l += 1
    return l
def fd2(d): return (d - (d & 1)) // 2
def wrapr(w, n):
    w = w + n if w < 0 else w
    return w - n if w >= n else w
class Geo:
    def __init__(g, SIG):
        g.SIG = SIG; g.LL = ell(SIG); g.H1 = g.LL + 1
        g.AWX = TX + 2 * SIG; g.AWY = TY + 2 * SIG; g.AGY = TY + 2 * GH; g.BWX = TX + 2 * g.H1
        g.A_NJ = g.AWX * g.AWY; g.B_NJ = 4 * g.BWX * TY
        g.A_G4 = 4 * g.AGY * (GWX // 4); g.B_G4 = 8 * TY * (GWX // 4) if STAGE_BG else 0
        g.O_BNJ = g.A_NJ; g.O_AG = g.A_NJ + g.B_NJ; g.O_BG = g.O_AG + g.A_G4; g.SIZE = g.O_BG + g.B_G4
    def zi(g, dz): return 0 if dz == -g.H1 else (1 if dz == -g.LL else (2 if dz == g.LL else 3))
    def dz_of(g, i): return [-g.H1, -g.LL, g.LL, g.H1][i]
def elements(SIG, PL):
    L = ell(SIG); out = []
    for SA, SB in ((1, 1), (1, -1)):
        for LA in (L, L + 1):
            for LB in (L, L + 1):
                a, b = SA * LA, SB * LB
                DX = 0 if PL == 2 else a
                DY = b if PL == 0 else (a if PL == 2 else 0)
                DZ = 0 if PL == 0 else b
                out.append((DX, DY, DZ))
    return out
def copy_region(lds, base, CNT, src_of):
    for thr in range(256):
        w64 = thr & ~63; lane = thr & 63
        for k in range((CNT + 255) // 256):
            i = thr + 256 * k
            if i < CNT:
                slot = base + 256 * k + w64 + lane
                assert slot == base + i
                lds[slot] = src_of(i)
def check(SIG, nx, ny, nz, hz):
    g = Geo(SIG); NF = nz + 2 * hz
    tnx, tny = nx // TX, ny // TY
    for (tx, ty) in {(0, 0), (tnx - 1, tny - 1), (tnx // 2, 0), (0, tny - 1)}:
        x0, y0 = tx * TX, ty * TY
        for zp in (hz, hz + nz - 1):
            lds = {}
            def njA(i):
                ry, rx = divmod(i, g.AWX)
                gx, gy = wrapr(x0 + rx - SIG, nx), wrapr(y0 + ry - SIG, ny)
                assert 0 <= gx < nx and 0 <= gy < ny
                return ('nj', gx, gy, zp)
            copy_region(lds, 0, g.A_NJ, njA)
            def njB(i):
                p, rem = divmod(i, g.BWX * TY); ry, rx = divmod(rem, g.BWX)
                gx = wrapr(x0 + rx - g.H1, nx); z = zp + g.dz_of(p)
                assert 0 <= gx < nx and 0 <= y0 + ry < ny and 0 <= z < NF
                return ('nj', gx, y0 + ry, z)
            copy_region(lds, g.O_BNJ, g.B_NJ, njB)
            R4 = GWX // 4
            def gA(i):
                slot, rem = divmod(i, g.AGY * R4); ry, c4 = divmod(rem, R4)
                gx, gy = wrapr(x0 - GH + 4 * c4, nx), wrapr(y0 + ry - GH, ny)
                assert gx % 4 == 0 and gx + 3 < nx and 0 <= gy < ny and slot < 4
                return ('G4', slot, gx, gy, zp)
            copy_region(lds, g.O_AG, g.A_G4, gA)
            def gB(i):
                c, rem = divmod(i, TY * R4); ry, c4 = divmod(rem, R4)
                dz = g.dz_of(c >> 1); slot = (c & 1) | ((dz & 1) << 2)
                gx = wrapr(x0 - GH + 4 * c4, nx); z = zp + fd2(dz)
                assert gx % 4 == 0 and gx + 3 < nx and 0 <= y0 + ry < ny and 0 <= z < NF and slot < 7
                return ('G4', slot, gx, y0 + ry, z)
            if STAGE_BG:
                copy_region(lds, g.O_BG, g.B_G4, gB)
            assert max(lds) < g.SIZE and min(lds) >= 0
            def gfloat(fi):   # float index into the LDS array viewed as floats
                e = lds[fi // 4]; assert e[0] == 'G4'
                return ('G', e[1], e[2] + fi % 4, e[3], e[4])
            for ly in range(TY):
                for lx in range(TX):
                    x, y = x0 + lx, y0 + ly
                    for DX, DY, DZ in [(SIG, 0, 0), (0, SIG, 0)] + elements(SIG, 0):
                        slot = (DX & 1) | ((DY & 1) << 1)
                        o = ly * g.AWX + lx
                        assert lds[o + (DY + SIG) * g.AWX + DX + SIG] == ('nj', wrapr(x + DX, nx), wrapr(y + DY, ny), zp)
                        assert lds[o + (SIG - DY) * g.AWX + SIG - DX] == ('nj', wrapr(x - DX, nx), wrapr(y - DY, ny), zp)
                        og = 4 * g.O_AG + slot * g.AGY * GWX + ly * GWX + lx
                        assert gfloat(og + (fd2(DY) + GH) * GWX + fd2(DX) + GH) == ('G', slot, wrapr(x + fd2(DX), nx), wrapr(y + fd2(DY), ny), zp)
                        assert gfloat(og + (fd2(-DY) + GH) * GWX + fd2(-DX) + GH) == ('G', slot, wrapr(x + fd2(-DX), nx), wrapr(y + fd2(-DY), ny), zp)
                    for DX, DY, DZ in elements(SIG, 1):
                        slot = (DX & 1) | ((DZ & 1) << 2)
                        cp, cm = 2 * g.zi(DZ) + (DX & 1), 2 * g.zi(-DZ) + (DX & 1)
                        o = g.O_BNJ + ly * g.BWX + lx + g.H1
                        assert lds[o + g.zi(DZ) * g.BWX * TY + DX] == ('nj', wrapr(x + DX, nx), y, zp + DZ)
                        assert lds[o + g.zi(-DZ) * g.BWX * TY - DX] == ('nj', wrapr(x - DX, nx), y, zp - DZ)
                        if STAGE_BG:
                            og = 4 * g.O_BG + ly * GWX + lx + GH
                            assert gfloat(og + cp * TY * GWX + fd2(DX)) == ('G', slot, wrapr(x + fd2(DX), nx), y, zp + fd2(DZ))
                            assert gfloat(og + cm * TY * GWX + fd2(-DX)) == ('G', slot, wrapr(x + fd2(-DX), nx), y, zp + fd2(-DZ))
    assert g.SIZE * 16 <= 60 * 1024 + (16 * 1024 if STAGE_BG else 0)


@pytest.mark.parametrize("sigma,nx,ny", [(2, 64, 4), (3, 64, 8), (5, 128, 12), (6, 64, 8), (8, 128, 12)])
def test_staged_collide_indexing(sigma, nx, ny):
    check(sigma, nx, ny, 2 * sigma + 4, sigma)
