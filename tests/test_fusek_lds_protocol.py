"""The LDS protocol of the multi-step kernel (k_sweepk), checked on the CPU.

A model of which LDS entries each step of a TX x TY tile writes and reads
over K steps, following the kernel's rules: step s runs on the tile grown
by K - s nodes; one plane per population over the window of step 2's
region (margin K - 2), indexed by the pulling node; a node of step s - 1
writes population i at its own position + e_i when that lies in step s's
region, and writes the wall rule of a link that crosses a non-periodic side
at its own position; a node of step s reads its own position in every
plane, or its fluid neighbour's for a wall node rebuilt by extrapolation.
For every tile of lattices from 1 x 1 up, with periodic, link-wise and
extrapolation sides, it checks: every access lies in the window, no entry
has two writers in a step, and every entry a step reads was written by the
step before it (with one buffer updated in place, an entry left from an
earlier step must not be read).  The built kernels (32 x 16 tiles with
K = 4 for the D2Q5 model and the flow alone, 32 x 8 tiles with K = 3 for
the D2Q9 thermal model) and the generic form with 64 x 8 tiles and K = 3 are
modelled.  No GPU is
used; the GPU tests check the values."""
import pytest

# (tile and K, temperature populations) of the built kernels, then the
# generic form with 64 x 8 tiles and K = 3
BUILT = [((32, 16, 4), 5), ((32, 16, 4), 0), ((32, 8, 3), 9)]
FORMS = BUILT + [((64, 8, 3), 5)]
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3


def _axis(v0, v, n, periodic):
    a = v0 + v
    if 0 <= a < n:
        return a
    return a % n if periodic else None


def _in_region(sx, sy, m, TX, TY):
    return -m <= sx < TX + m and -m <= sy < TY + m


def _directions(ng):
    """(plane, direction) of every population: 9 flow, then ng temperature."""
    return [(i, i) for i in range(9)] + [(9 + j, j) for j in range(ng)]


def _tile_protocol(shape, nx, ny, px, py, nee, ng, x0, y0):
    TX, TY, K = shape
    WM = K - 2
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
                if _in_region(*t, m_next, TX, TY):
                    pos.append((p, t))
            if wall_node(x, y) and _in_region(sx, sy, m_next, TX, TY):
                for i in range(1, 9):
                    ax, ay = x - EX[i], y - EY[i]
                    crosses = (EY[i] and not (0 <= ay < ny) and not py) or (EX[i] and not (0 <= ax < nx) and not px)
                    if crosses:
                        pos.append((i, (sx, sy)))
                        if i < ng:
                            pos.append((9 + i, (sx, sy)))
            for e in pos:
                p, (tx, ty) = e
                assert 0 <= p < np_ and _in_region(tx, ty, WM, TX, TY), ("write outside the window", e)
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
                assert _in_region(*at, WM, TX, TY), ("read outside the window", p, at, (sx, sy))
                out.append((p, at))
        return out

    counts = []
    prev = None
    for s in range(1, K + 1):
        m = K - s
        if s < K:
            nodes = list(step_nodes(m))
        else:
            nodes = [(ix, iy, x0 + ix, y0 + iy) for iy in range(TY) for ix in range(TX)
                     if x0 + ix < nx and y0 + iy < ny]
        if prev is not None:
            for e in reads(nodes):
                assert e in prev, ("step reads an entry the step before did not write", s, e)
        if s < K:
            prev = writes(m - 1, nodes)
        counts.append(len(nodes))
    return counts


def _cases(shape, ng):
    TX, TY, _ = shape
    sizes = [(1, 1), (1, 6), (7, 1), (2, 2), (3, 7), (2, 11), (33, 3), (32, 16), (34, 17), (65, 3), (64, 8),
             (66, 9), (129, 17), (70, 45), (130, 70), (200, 33)]
    if (shape, ng) not in BUILT:
        # the generic form, not built: lattices up to a few tiles
        sizes = [sz for sz in sizes if sz[0] * sz[1] <= 129 * 17]
    for nx, ny in sizes:
        for px in (False, True):
            for py in (False, True):
                yield shape, ng, nx, ny, px, py, (False,) * 4
                # extrapolation walls on the non-periodic sides, where the
                # launch allows them (no one-node last tile on such an axis)
                nee = (not px and nx % TX != 1 and nx >= 3, not px and nx % TX != 1 and nx >= 3,
                       not py and ny % TY != 1 and ny >= 3, not py and ny % TY != 1 and ny >= 3)
                if any(nee):
                    yield shape, ng, nx, ny, px, py, nee


@pytest.mark.parametrize("shape,ng,nx,ny,px,py,nee", [c for sh, ng in FORMS for c in _cases(sh, ng)])
def test_multi_step_lds_protocol(shape, ng, nx, ny, px, py, nee):
    TX, TY, K = shape
    total = None
    for y0 in range(0, ny, TY):
        for x0 in range(0, nx, TX):
            counts = _tile_protocol(shape, nx, ny, px, py, nee, ng, x0, y0)
            total = counts if total is None else [a + b for a, b in zip(total, counts)]
    # the last step covers every node once
    assert total[-1] == nx * ny
    if K == 4 and not px and not py:
        # collisions per launch of an open interior tile: sum over the
        # steps of (TX + 2m)(TY + 2m), m = 3, 2, 1, 0
        if nx >= 3 * TX and ny >= 3 * TY:
            c = _tile_protocol(shape, nx, ny, px, py, nee, ng, TX, TY)
            assert sum(c) == sum((TX + 2 * m) * (TY + 2 * m) for m in range(K))


@pytest.mark.parametrize("shape", sorted({sh for sh, _ in FORMS}))
def test_one_node_edge_tile_breaks_extrapolation(shape):
    """Why the launch falls back to single steps when a lattice with walls
    by extrapolation leaves a one-node last tile: the wall node's fluid
    neighbour lies outside the step's region."""
    TX = shape[0]
    with pytest.raises(AssertionError):
        for x0 in range(0, 2 * TX + 1, TX):
            _tile_protocol(shape, 2 * TX + 1, 20, False, True, (True, True, False, False), 5, x0, 0)
