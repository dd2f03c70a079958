"""In-place (AA) streaming index maps, checked on the CPU.

A model of the two maps the in-place D2Q9 step uses: where the value f_i of
node x at time t sits (the read map, by parity of t) and where a node puts
its post-collision f*_i for the next step's reader (the write map).  On
small lattices with every wall combination the maps must (i) give each slot
exactly one reader and one writer per step, that writer being its reader
(no ordering between nodes is needed), and (ii) reproduce two-buffer pull
streaming with halfway bounce-back exactly, for an arbitrary node- and
time-dependent collision.  The GPU tests check the kernels themselves
(bitwise against the two-buffer path).
"""
import itertools

import numpy as np
import pytest

C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def read_slot(i, x, y, nx, ny, walls, mode):
    """Slot holding f_i(x, y): mode 0 two buffers (post-collision values at
    their writer), 1 in place at even t, 2 in place at odd t."""
    N = nx * ny
    if mode == 1:
        return i * N + y * nx + x
    s, n, bounce = [x - C[i][0], y - C[i][1]], [nx, ny], False
    for a in range(2):
        if C[i][a] != 0 and not 0 <= s[a] < n[a]:
            if walls & (1 << a):
                bounce = True
            else:
                s[a] = n[a] - 1 if s[a] < 0 else 0
    j = OPP[i] if mode == 2 else i
    if bounce:
        return OPP[j] * N + y * nx + x
    return j * N + s[1] * nx + s[0]


def write_slot(i, x, y, nx, ny, walls, mode):
    """Slot that receives f*_i of (x, y) in an in-place step of `mode`."""
    N, n, o = nx * ny, y * nx + x, OPP[i]
    if mode == 1:
        return o * N + n
    tx, ty = x + C[i][0], y + C[i][1]
    if (walls & 1 and not 0 <= tx < nx) or (walls & 2 and not 0 <= ty < ny):
        return o * N + n
    return i * N + (ty % ny) * nx + (tx % nx)


def collide(f, x, y, t):
    return [v * 1.0001 + 0.37 * ((7 * x + 3 * y + i + t) % 5) for i, v in enumerate(f)]


CASES = [(nx, ny, w) for nx, ny, w in itertools.product([1, 2, 3, 5], [1, 2, 4], range(4))
         if not (w & 1 and nx < 2) and not (w & 2 and ny < 2)]


@pytest.mark.parametrize("nx,ny,walls", CASES)
def test_in_place_maps_are_race_free_and_equal_two_buffer_streaming(nx, ny, walls):
    N = nx * ny
    f0 = np.random.default_rng(100 * nx + 10 * ny + walls).normal(size=(9, N))
    two = np.full(9 * N, np.nan)
    one = np.full(9 * N, np.nan)
    for y, x, i in itertools.product(range(ny), range(nx), range(9)):
        two[read_slot(i, x, y, nx, ny, walls, 0)] = f0[i, y * nx + x]
        one[read_slot(i, x, y, nx, ny, walls, 1)] = f0[i, y * nx + x]
    assert not np.isnan(two).any() and not np.isnan(one).any()
    for t in range(6):
        nxt = np.full(9 * N, np.nan)
        for y, x in itertools.product(range(ny), range(nx)):
            fs = collide([two[read_slot(i, x, y, nx, ny, walls, 0)] for i in range(9)], x, y, t)
            for i in range(9):
                nxt[i * N + y * nx + x] = fs[i]
        two = nxt
        mode = 1 if t % 2 == 0 else 2
        reader, writer, new = {}, {}, one.copy()
        for y, x in itertools.product(range(ny), range(nx)):
            n, f = y * nx + x, []
            for i in range(9):
                k = read_slot(i, x, y, nx, ny, walls, mode)
                assert reader.setdefault(k, n) == n
                f.append(one[k])
            for i, v in enumerate(collide(f, x, y, t)):
                k = write_slot(i, x, y, nx, ny, walls, mode)
                assert writer.setdefault(k, n) == n
                new[k] = v
        assert len(reader) == len(writer) == 9 * N
        assert all(reader[k] == writer[k] for k in writer)
        one = new
        nm = 1 if (t + 1) % 2 == 0 else 2
        for y, x, i in itertools.product(range(ny), range(nx), range(9)):
            assert two[read_slot(i, x, y, nx, ny, walls, 0)] == \
                one[read_slot(i, x, y, nx, ny, walls, nm)], (t, x, y, i)


# ---------------------------------------------------------------- D3Q19
# The same two maps for the 19 velocities (order of App. A; opposite pairs
# (2k-1, 2k)), with walls on any subset of the three axes: the in-place
# velocity pass (aa3d.h) reads through pull_index, the z-march uses them in
# pair form (below).
C3 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
      (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
      (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
OPP3 = [0] + [k + 1 if k % 2 else k - 1 for k in range(1, 19)]


def read_slot3(i, p, n, walls, mode):
    N = n[0] * n[1] * n[2]
    node = lambda q: (q[2] * n[1] + q[1]) * n[0] + q[0]
    if mode == 1:
        return i * N + node(p)
    s, bounce = [p[a] - C3[i][a] for a in range(3)], False
    for a in range(3):
        if C3[i][a] != 0 and not 0 <= s[a] < n[a]:
            if walls & (1 << a):
                bounce = True
            else:
                s[a] = n[a] - 1 if s[a] < 0 else 0
    j = OPP3[i] if mode == 2 else i
    if bounce:
        return OPP3[j] * N + node(p)
    return j * N + node(s)


def write_slot3(i, p, n, walls, mode):
    N = n[0] * n[1] * n[2]
    node = lambda q: (q[2] * n[1] + q[1]) * n[0] + q[0]
    o = OPP3[i]
    if mode == 1:
        return o * N + node(p)
    t = [p[a] + C3[i][a] for a in range(3)]
    if any(walls & (1 << a) and not 0 <= t[a] < n[a] for a in range(3)):
        return o * N + node(p)
    return i * N + node([t[a] % n[a] for a in range(3)])


CASES3 = [(n, w) for n, w in itertools.product([(1, 2, 3), (2, 2, 2), (3, 2, 4), (2, 3, 1)],
                                               range(8))
          if all(not (w & (1 << a)) or n[a] >= 2 for a in range(3))]


def test_d3q19_opposites():
    assert all(tuple(-c for c in C3[i]) == C3[OPP3[i]] for i in range(19))


@pytest.mark.parametrize("n,walls", CASES3)
def test_d3q19_in_place_maps_are_race_free_and_equal_two_buffer_streaming(n, walls):
    N = n[0] * n[1] * n[2]
    nodes = list(itertools.product(range(n[0]), range(n[1]), range(n[2])))
    f0 = np.random.default_rng(sum(n) + 10 * walls).normal(size=(19, N))
    two = np.full(19 * N, np.nan)
    one = np.full(19 * N, np.nan)
    idx = lambda p: (p[2] * n[1] + p[1]) * n[0] + p[0]
    for p, i in itertools.product(nodes, range(19)):
        two[read_slot3(i, p, n, walls, 0)] = f0[i, idx(p)]
        one[read_slot3(i, p, n, walls, 1)] = f0[i, idx(p)]
    assert not np.isnan(two).any() and not np.isnan(one).any()
    for t in range(4):
        nxt = np.full(19 * N, np.nan)
        for p in nodes:
            fs = [v * 1.0001 + 0.37 * ((7 * p[0] + 3 * p[1] + 5 * p[2] + i + t) % 5)
                  for i, v in enumerate(two[read_slot3(i, p, n, walls, 0)] for i in range(19))]
            for i in range(19):
                nxt[i * N + idx(p)] = fs[i]
        two = nxt
        mode = 1 if t % 2 == 0 else 2
        reader, writer, new = {}, {}, one.copy()
        for p in nodes:
            f = []
            for i in range(19):
                k = read_slot3(i, p, n, walls, mode)
                assert reader.setdefault(k, idx(p)) == idx(p)
                f.append(one[k])
            fs = [v * 1.0001 + 0.37 * ((7 * p[0] + 3 * p[1] + 5 * p[2] + i + t) % 5)
                  for i, v in enumerate(f)]
            for i, v in enumerate(fs):
                k = write_slot3(i, p, n, walls, mode)
                assert writer.setdefault(k, idx(p)) == idx(p)
                new[k] = v
        assert len(reader) == len(writer) == 19 * N
        assert all(reader[k] == writer[k] for k in writer)
        one = new
        nm = 1 if (t + 1) % 2 == 0 else 2
        for p, i in itertools.product(nodes, range(19)):
            assert two[read_slot3(i, p, n, walls, 0)] == one[read_slot3(i, p, n, walls, nm)], \
                (t, p, i)


# ------------------------------------------------- the maps in pair form
# The D3Q19 z-march handles a node with two lanes: lane s holds member s of
# each opposite pair K (direction 2K - 1 + s) and addresses the pair's two
# planes with an offset member * N + node.  Its pull geometry swaps the
# neighbour deltas with s, the two-buffer pull is pair_src, and the in-place
# maps swap members (step3d.h: make_pair_pull, pair_src, aa_pair_src,
# aa_pair_dst).  This model follows that code and must give, slot for slot,
# the direct maps above (and the two-buffer pull of read_slot3 mode 0).
def make_pair_pull(p, s, n, walls):
    stride = (1, n[0], n[0] * n[1])
    q = dict(dm=[0] * 3, dp=[0] * 3, wm=[False] * 3, wp=[False] * 3)
    for a in range(3):
        wall = bool(walls & (1 << a))
        lo, hi = wall and p[a] == 0, wall and p[a] == n[a] - 1
        from_minus = (n[a] - 1 if p[a] == 0 else -1) * stride[a]
        from_plus = (1 - n[a] if p[a] == n[a] - 1 else 1) * stride[a]
        q["dm"][a], q["dp"][a] = (from_plus, from_minus) if s else (from_minus, from_plus)
        q["wm"][a], q["wp"][a] = (hi, lo) if s else (lo, hi)
    q["self"] = (p[2] * n[1] + p[1]) * n[0] + p[0]
    return q


def pair_src(q, K, s, N, walls):
    c = C3[2 * K - 1]
    off = q["self"]
    bounce = False
    for a in range(3):
        if c[a] > 0:
            off += q["dm"][a]
            bounce |= q["wm"][a]
        elif c[a] < 0:
            off += q["dp"][a]
            bounce |= q["wp"][a]
    if walls and bounce:
        return (0 if s else N) + q["self"]
    return (N if s else 0) + off


def swap_members(o, N):
    return o - N if o >= N else o + N


def aa_pair_src(q, K, s, aa, N, walls):
    if aa == 1:
        return (N if s else 0) + q["self"]
    return swap_members(pair_src(q, K, s, N, walls), N)


def aa_pair_dst(q, K, s, aa, N, walls):
    if aa == 1:
        return (0 if s else N) + q["self"]
    r = dict(q, dm=list(q["dp"]), dp=list(q["dm"]), wm=list(q["wp"]), wp=list(q["wm"]))
    return swap_members(pair_src(r, K, 1 - s, N, walls), N)


def slot_of(K, o, N):
    """(direction, node) of a pair offset: member o // N of pair K."""
    return (2 * K - 1 + o // N) * N + o % N


@pytest.mark.parametrize("n,walls", CASES3)
def test_d3q19_pair_maps_equal_the_slot_maps(n, walls):
    N = n[0] * n[1] * n[2]
    for p in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        for s in (0, 1):
            q = make_pair_pull(p, s, n, walls)
            for K in range(1, 10):
                i = 2 * K - 1 + s
                assert slot_of(K, pair_src(q, K, s, N, walls), N) == \
                    read_slot3(i, p, n, walls, 0), (p, s, K)
                for aa in (1, 2):
                    assert slot_of(K, aa_pair_src(q, K, s, aa, N, walls), N) == \
                        read_slot3(i, p, n, walls, aa), (p, s, K, aa)
                    assert slot_of(K, aa_pair_dst(q, K, s, aa, N, walls), N) == \
                        write_slot3(i, p, n, walls, aa), (p, s, K, aa)
