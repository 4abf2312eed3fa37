"""The LDS protocol of the three-step kernel (k_sweepk), checked on the CPU.

A model of which LDS entries each step of a 64 x 8 tile writes and reads,
following the kernel's rules: step 1 runs on the tile grown by two nodes,
step 2 on the tile grown by one, step 3 on the tile; one plane per
population over the window of step 2's region, indexed by the pulling node;
a node of step s - 1 writes population i at its own position + e_i when
that lies in step s's region, and writes the wall rule of a link that
crosses a non-periodic side at its own position; a node of step s reads its
own position in every plane, or its fluid neighbour's for a wall node
rebuilt by extrapolation.  For every tile of lattices from 1 x 1 up, with
periodic, link-wise and extrapolation sides, both variants are checked:
every access lies in the window, no entry has two writers in a step, and
every entry a step reads was written by the step before it (with one
buffer updated in place, an entry left from step 1 must not be read by
step 3).  No GPU is used; the GPU tests check the values."""
import pytest

TX, TY, K = 64, 8, 3
WM = K - 2
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3


def _axis(v0, v, n, periodic):
    a = v0 + v
    if 0 <= a < n:
        return a
    return a % n if periodic else None


def _in_region(sx, sy, m):
    return -m <= sx < TX + m and -m <= sy < TY + m


def _directions(ng):
    """(plane, direction) of every population: 9 flow, then ng temperature."""
    return [(i, i) for i in range(9)] + [(9 + j, j) for j in range(ng)]


def _tile_protocol(nx, ny, px, py, nee, ng, x0, y0):
    planes = _directions(ng)
    np_ = 9 + ng

    def wall_node(x, y):
        return (not px and (x == 0 or x == nx - 1)) or (not py and (y == 0 or y == ny - 1))

    def nee_node(x, y):
        return (nee[LEFT] and x == 0) or (nee[RIGHT] and x == nx - 1) or (nee[BOTTOM] and y == 0) or \
            (nee[TOP] and y == ny - 1)

    def step_nodes(m):
        for sy in range(-m, TY + m):
            for sx in range(-m, TX + m):
                x, y = _axis(x0, sx, nx, px), _axis(y0, sy, ny, py)
                if x is not None and y is not None:
                    yield sx, sy, x, y

    def writes(m_next, nodes):
        out = {}
        for sx, sy, x, y in nodes:
            pos = []
            for p, i in planes:
                t = (sx + EX[i], sy + EY[i])
                if _in_region(*t, m_next):
                    pos.append((p, t))
            if wall_node(x, y) and _in_region(sx, sy, m_next):
                for i in range(1, 9):
                    ax, ay = x - EX[i], y - EY[i]
                    crosses = (EY[i] and not (0 <= ay < ny) and not py) or (EX[i] and not (0 <= ax < nx) and not px)
                    if crosses:
                        pos.append((i, (sx, sy)))
                        if i < ng:
                            pos.append((9 + i, (sx, sy)))
            for e in pos:
                p, (tx, ty) = e
                assert 0 <= p < np_ and _in_region(tx, ty, WM), ("write outside the window", e)
                assert e not in out, ("two writers", e, out.get(e), (sx, sy))
                out[e] = (sx, sy)
        return out

    def reads(nodes):
        out = []
        for sx, sy, x, y in nodes:
            at = (sx, sy)
            if nee_node(x, y):
                onl, onr = nee[LEFT] and x == 0, nee[RIGHT] and x == nx - 1
                onb, ont = nee[BOTTOM] and y == 0, nee[TOP] and y == ny - 1
                fx = x + (1 if onl else (-1 if onr else 0))
                fy = y + (1 if onb else (-1 if ont else 0))
                at = (sx + fx - x, sy + fy - y)
            for p in range(np_):
                assert _in_region(*at, WM), ("read outside the window", p, at, (sx, sy))
                out.append((p, at))
        return out

    step1 = list(step_nodes(WM + 1))
    step2 = list(step_nodes(WM))
    step3 = [(ix, iy, x0 + ix, y0 + iy) for iy in range(TY) for ix in range(TX)
             if x0 + ix < nx and y0 + iy < ny]
    w1 = writes(WM, step1)
    for e in reads(step2):
        assert e in w1, ("step 2 reads an entry step 1 did not write", e)
    w2 = writes(0, step2)
    for e in reads(step3):
        assert e in w2, ("step 3 reads an entry step 2 did not write", e)
    return len(step1), len(step2), len(step3)


def _cases():
    sizes = [(1, 1), (1, 6), (7, 1), (2, 2), (3, 7), (2, 11), (65, 3), (64, 8), (66, 9), (129, 17), (70, 45),
             (130, 70), (200, 33)]
    for nx, ny in sizes:
        for px in (False, True):
            for py in (False, True):
                yield nx, ny, px, py, (False,) * 4
                # extrapolation walls on the non-periodic sides, where the
                # launch allows them (no one-node last tile on such an axis)
                nee = (not px and nx % TX != 1 and nx >= 3, not px and nx % TX != 1 and nx >= 3,
                       not py and ny % TY != 1 and ny >= 3, not py and ny % TY != 1 and ny >= 3)
                if any(nee):
                    yield nx, ny, px, py, nee


@pytest.mark.parametrize("ng", [5, 0])
@pytest.mark.parametrize("nx,ny,px,py,nee", list(_cases()))
def test_three_step_lds_protocol(nx, ny, px, py, nee, ng):
    total = [0, 0, 0]
    for y0 in range(0, ny, TY):
        for x0 in range(0, nx, TX):
            counts = _tile_protocol(nx, ny, px, py, nee, ng, x0, y0)
            total = [a + b for a, b in zip(total, counts)]
    # the last step covers every node once
    assert total[2] == nx * ny


def test_one_node_edge_tile_breaks_extrapolation():
    """Why the launch falls back to single steps when a lattice with walls
    by extrapolation leaves a one-node last tile: the wall node's fluid
    neighbour lies outside the step's region."""
    with pytest.raises(AssertionError):
        for x0 in range(0, 129, TX):
            _tile_protocol(129, 12, False, True, (True, True, False, False), 5, x0, 0)
