"""The in-place AA addressing with walls, checked on the CPU.

The library keeps one population array and updates it in place: an even
sweep reads a cell's own slots and writes its post-collision values into
its own opposite slots (or into a mailbox slot of a ghost cell), an odd
sweep gathers from neighbours' slots and scatters into neighbours' slots
(csrc/lbm_sweep_dev.h, update_cell).  Walls change where a population is
read and written: resting no-slip walls on the x and y faces use the
cell's own slots, free-slip walls reflect into the slot of the tangential
neighbour, no-slip z walls use the ghost-plane mailbox.

This test restates that slot addressing in numpy and checks, for every
wall combination, that (a) within one sweep no slot is touched by two
cells, so the sweep is race-free in any order, and (b) an
even and an odd sweep done cell by cell in random order, with the identity
in place of the collision, move every population where plain two-lattice
streaming with bounce-back (Eq. BBBC) and specular reflection (Eq.
FreeSlipBC) puts it.  The device kernels themselves are checked against the
oracle by the GPU parity tests; this pins the addressing scheme they
implement."""
import numpy as np
import pytest

# the library's velocity order: rest, nine directions, their opposites nine apart
CX = [0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0]
CY = [0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1]
CZ = [0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1]
Q = 19
OPP = [0] + [q + 9 for q in range(1, 10)] + [q - 9 for q in range(10, 19)]
DIR = {(CX[q], CY[q], CZ[q]): q for q in range(Q)}


def refl(q, m):
    """Direction q with the components flagged in m (bit 0 x, 1 y, 2 z) reversed."""
    e = [CX[q], CY[q], CZ[q]]
    for k in range(3):
        if m >> k & 1:
            e[k] = -e[k]
    return DIR[tuple(e)]


class Box:
    def __init__(self, n, xw, yw, zper, zs):
        self.nx, self.ny, self.nz = n
        self.xw, self.yw, self.zper, self.zs = xw, yw, zper, zs
        self.nxy = self.nx * self.ny

    def idx(self, x, y, z):
        """Plane-shifted cell index (planes 0 and nz + 1 are the ghost planes)."""
        return (z + 1) * self.nxy + (y % self.ny) * self.nx + (x % self.nx)

    def wrapz(self, z):
        return z % self.nz if self.zper else z

    def crossing(self, x, y, z, e, outgoing):
        """Walls crossed by a population leaving (outgoing) or arriving along e."""
        s = 1 if outgoing else -1
        bx = self.xw and (x + s * e[0] < 0 or x + s * e[0] >= self.nx)
        by = self.yw and (y + s * e[1] < 0 or y + s * e[1] >= self.ny)
        bz = not self.zper and (z + s * e[2] < 0 or z + s * e[2] >= self.nz)
        return bx, by, bz

    # ------------------------------------------------------------ the sweeps
    def even_slots(self, x, y, z):
        """(reads, writes): reads [(q, slot)], writes [(q_from, slot)]."""
        own = self.idx(x, y, z)
        reads = [(q, (q, own)) for q in range(Q)]
        writes = []
        for q in range(Q):
            e = (CX[q], CY[q], CZ[q])
            bx, by, bz = self.crossing(x, y, z, e, True)
            if bz and not self.zs:        # no-slip z wall: mailbox in the ghost plane
                writes.append((q, (q, self.idx(x + e[0], y + e[1], z + e[2]))))
            else:                         # streaming, side walls, reflections: own slot
                writes.append((q, (OPP[q], own)))
        return reads, writes

    def odd_slots(self, x, y, z):
        own = self.idx(x, y, z)
        reads, writes = [], []
        for q in range(Q):
            e = (CX[q], CY[q], CZ[q])
            # gather of direction q
            ix, iy, iz = self.crossing(x, y, z, e, False)
            nsz = iz and not self.zs
            if nsz:
                ix = iy = iz = False
            if (ix and self.xw == 1) or (iy and self.yw == 1):
                reads.append((q, (q, own)))
            elif ix or iy or iz:
                m = ix | iy << 1 | iz << 2
                t = [0 if ix else e[0], 0 if iy else e[1], 0 if iz else e[2]]
                reads.append((q, (OPP[refl(q, m)], self.idx(x - t[0], y - t[1], self.wrapz(z - t[2])))))
            else:
                reads.append((q, (OPP[q], self.idx(x - e[0], y - e[1], self.wrapz(z - e[2]) if self.zper else z - e[2]))))
            # scatter of direction q
            ox, oy, oz = self.crossing(x, y, z, e, True)
            to_wall = oz and not self.zs
            to_side = not to_wall and ((ox and self.xw == 1) or (oy and self.yw == 1))
            to_slip = not to_wall and not to_side and (ox or oy or oz)
            if to_slip:
                m = ox | oy << 1 | oz << 2
                t = [0 if ox else e[0], 0 if oy else e[1], 0 if oz else e[2]]
                writes.append((q, (refl(q, m), self.idx(x + t[0], y + t[1], self.wrapz(z + t[2])))))
            elif to_wall or to_side:
                writes.append((q, (OPP[q], own)))
            else:
                writes.append((q, (q, self.idx(x + e[0], y + e[1], self.wrapz(z + e[2])))))
        return reads, writes

    def cells(self):
        return [(x, y, z) for z in range(self.nz) for y in range(self.ny) for x in range(self.nx)]

    # ------------------------------------------------------------ reference
    def stream_reference(self, f):
        """Two-lattice streaming of natural-layout populations f[q][z][y][x]
        with bounce-back and specular reflection (identity collision)."""
        g = np.full_like(f, np.nan)
        for (x, y, z) in self.cells():
            for q in range(Q):
                e = (CX[q], CY[q], CZ[q])
                bx, by, bz = self.crossing(x, y, z, e, True)
                if (bz and not self.zs) or (bx and self.xw == 1) or (by and self.yw == 1):
                    g[OPP[q], z, y, x] = f[q, z, y, x]
                elif bx or by or bz:
                    m = bx | by << 1 | bz << 2
                    dx, dy, dz = (x if bx else (x + e[0]) % self.nx, y if by else (y + e[1]) % self.ny,
                                  z if bz else (z + e[2]) % self.nz)
                    g[refl(q, m), dz, dy, dx] = f[q, z, y, x]
                else:
                    g[q, (z + e[2]) % self.nz, (y + e[1]) % self.ny, (x + e[0]) % self.nx] = f[q, z, y, x]
        return g


CASES = {
    "periodic": (0, 0, True, False),
    "moving z walls": (0, 0, False, False),
    "no-slip x, y": (1, 1, True, False),
    "free-slip x": (2, 0, True, False),
    "free-slip x, y": (2, 2, True, False),
    "free-slip everywhere": (2, 2, False, True),
    "free-slip x, no-slip y": (2, 1, True, False),
    "no-slip x, free-slip z": (1, 0, False, True),
    "free-slip y, moving z": (0, 2, False, False),
    "no-slip x, y, moving z": (1, 1, False, False),
}


def _slot_owners(box, sweep):
    """{slot: cell} of the reads and of the writes of one sweep; a slot that
    two cells read, or two cells write, fails."""
    rd, wr = {}, {}
    for c in box.cells():
        reads, writes = sweep(*c)
        assert len({q for q, _ in reads}) == Q and len({q for q, _ in writes}) == Q, (sweep.__name__, c)
        for own, lst in ((rd, reads), (wr, writes)):
            slots = [s for _, s in lst]
            assert len(set(slots)) == Q, (sweep.__name__, c)
            for s in slots:
                assert s not in own, (sweep.__name__, c, s, own.get(s))
                own[s] = c
    return rd, wr


@pytest.mark.parametrize("case", list(CASES))
def test_each_sweep_is_race_free_and_the_pair_closes(case):
    """Within a sweep no slot is read or written by two cells, and no slot
    that one cell reads is written by another, so the cells can run in any
    order; every slot the odd sweep reads was written by the even sweep, and
    the odd sweep writes every natural slot the next even sweep reads."""
    box = Box((5, 4, 3), *CASES[case])
    ev_r, ev_w = _slot_owners(box, box.even_slots)
    od_r, od_w = _slot_owners(box, box.odd_slots)
    for rd, wr, name in ((ev_r, ev_w, "even"), (od_r, od_w, "odd")):
        for s in rd.keys() & wr.keys():
            assert rd[s] == wr[s], (case, name, s, rd[s], wr[s])
    assert od_r.keys() <= ev_w.keys(), (case, sorted(od_r.keys() - ev_w.keys())[:4])
    assert ev_r.keys() <= od_w.keys(), (case, sorted(ev_r.keys() - od_w.keys())[:4])
    if box.zper or box.zs:   # no ghost plane in use: the sweeps stay in the cells' own slots
        assert ev_r.keys() == ev_w.keys() == od_r.keys() == od_w.keys()


@pytest.mark.parametrize("case", list(CASES))
def test_even_odd_pair_in_random_order_equals_two_lattice_streaming(case):
    box = Box((5, 4, 3), *CASES[case])
    rng = np.random.default_rng(len(case))
    f0 = rng.standard_normal((Q, box.nz, box.ny, box.nx))
    A = np.full((Q, (box.nz + 2) * box.nxy), np.nan)
    for (x, y, z) in box.cells():
        A[:, box.idx(x, y, z)] = f0[:, z, y, x]
    cells = box.cells()
    for sweep in (box.even_slots, box.odd_slots):
        for k in rng.permutation(len(cells)):
            reads, writes = sweep(*cells[k])
            v = {q: A[s] for q, s in reads}                   # gather (identity collision)
            for q, s in writes:
                A[s] = v[q]
    # after the pair the natural slots hold the populations of two streaming steps
    ref = box.stream_reference(box.stream_reference(f0))
    got = np.array([[A[q, box.idx(x, y, z)] for (x, y, z) in cells] for q in range(Q)])
    want = np.array([[ref[q, z, y, x] for (x, y, z) in cells] for q in range(Q)])
    np.testing.assert_array_equal(got, want)
