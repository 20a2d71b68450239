"""The product with the packed symmetric moment matrix, its scheme checked on
the CPU.

The slender-body solve (Sec. 3) multiplies by the dense moment matrix in
every GMRES iteration.  The matrix is symmetric, so the library stores only
its upper triangle of 64 x 64 tiles, row-major (csrc/sbf.hip): tile (i, j),
i <= j, starts at tile number i (2 nt - i + 1)/2 + j - i; a diagonal tile
holds its whole symmetric block.  One workgroup takes a chunk of up to 8
consecutive tiles of one tile row i and writes (a) the chunk's row sums
T x_j into slot i + c of block i (c: the chunk's index in its row) and
(b) for every off-diagonal tile the column sums T^T x_i into slot i of
block j.  A second pass adds, for block b, the slots 0 .. b + ceil((nt -
b)/8) - 1.  This restates that plan in numpy and checks that the packing
is a bijection, that every slot the second pass reads is written by exactly
one workgroup (nothing stale is read, nothing is written twice), and that
the sum equals the full matrix product, on ragged orders that span several
chunks per tile row.  The device kernels are checked against the FP64
reference by the GPU parity tests; this pins the plan they follow."""
import numpy as np
import pytest

TS, SG = 64, 8


def tile_number(i, j, nt):
    return i * (2 * nt - i + 1) // 2 + (j - i)


def chunks(nt):
    """(i, j0, ng, slot) per workgroup."""
    out = []
    for i in range(nt):
        for c, j0 in enumerate(range(i, nt, SG)):
            out.append((i, j0, min(SG, nt - j0), i + c))
    return out


def packed(A, nt):
    Dp = nt * TS
    P = np.zeros((Dp, Dp))
    P[:A.shape[0], :A.shape[1]] = A
    W = np.zeros((nt * (nt + 1) // 2, TS, TS))
    for i in range(nt):
        for j in range(i, nt):
            W[tile_number(i, j, nt)] = P[i * TS:(i + 1) * TS, j * TS:(j + 1) * TS]
    return W


def product(W, x, nt, D, plan=None):
    xp = np.zeros(nt * TS)
    xp[:D] = x
    part = np.full((nt, nt * TS), np.nan)     # slots x rows; NaN marks a slot nobody wrote
    writer = {}
    for k, (i, j0, ng, slot) in enumerate(chunks(nt) if plan is None else plan):
        rows = np.zeros(TS)
        xi = xp[i * TS:(i + 1) * TS]
        for j in range(j0, j0 + ng):
            T = W[tile_number(i, j, nt)]
            rows += T @ xp[j * TS:(j + 1) * TS]
            if j != i:
                assert (i, j) not in writer, ("column sums written twice", i, j)
                writer[(i, j)] = k
                part[i, j * TS:(j + 1) * TS] = T.T @ xi
        assert (slot, i) not in writer, ("row sums written twice", slot, i)
        writer[(slot, i)] = k
        part[slot, i * TS:(i + 1) * TS] = rows
    y = np.zeros(nt * TS)
    for b in range(nt):
        ns = b + -(-(nt - b) // SG)
        assert ns <= nt                        # slots fit the nt x nt x 64 buffer
        blk = part[:ns, b * TS:(b + 1) * TS]
        assert not np.isnan(blk).any(), ("stale slot read", b)
        # every slot written for block b is read
        assert all(s < ns for (s, bb) in writer if bb == b), b
        y[b * TS:(b + 1) * TS] = blk.sum(axis=0)
    return y[:D]


@pytest.mark.parametrize("nt", [1, 2, 7, 8, 9, 17, 24])
def test_packed_tile_numbering_is_a_bijection(nt):
    seen = sorted(tile_number(i, j, nt) for i in range(nt) for j in range(i, nt))
    assert seen == list(range(nt * (nt + 1) // 2))


@pytest.mark.parametrize("D", [1, 63, 64, 65, 18 * 37, 1100, 64 * 17 + 5])
def test_chunked_symmetric_product_equals_the_full_product(D):
    nt = -(-D // TS)
    rng = np.random.default_rng(D)
    B = rng.standard_normal((D, D))
    A = B + B.T
    x = rng.standard_normal(D)
    y = product(packed(A, nt), x, nt, D)
    want = A @ x
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-12 * np.abs(A).sum(axis=1).max() * np.abs(x).max())


@pytest.mark.parametrize("mistake", ["diagonal tiles only", "one slot per tile row"])
def test_planted_plan_mistakes_are_caught(mistake):
    """A plan that drops the off-diagonal tiles leaves slots of the second
    pass unwritten; one that gives every chunk of a tile row the same slot
    writes a slot twice."""
    nt = 10
    D = nt * TS - 3
    rng = np.random.default_rng(2)
    B = rng.standard_normal((D, D))
    W = packed(B + B.T, nt)
    if mistake == "diagonal tiles only":
        plan = [(i, i, 1, i) for i in range(nt)]
    else:
        plan = [(i, j0, ng, i) for (i, j0, ng, _) in chunks(nt)]
    with pytest.raises(AssertionError):
        product(W, rng.standard_normal(D), nt, D, plan)
