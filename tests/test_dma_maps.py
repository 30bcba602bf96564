"""CPU replica of the LDS-DMA maps of the streaming GEMM kernels.

The streaming core and the short-reduction kernel copy operands from global
memory into LDS with global_load_lds: lane i of a DMA instruction writes
LDS address base + i * unit, so each operand layout is defined by which
global element each slot (instruction * 64 + lane) copies, and read back by
its fragment functions.  These tests restate those formulas (lane_off,
k_of, frag, frag4, rbase/clamp of the operand types, the short-reduction
kernel's per-wave DMA offsets and its vmcnt wait counts) in Python and
check, for every tile shape the launchers use and the operand shapes of
every workload:

* each stage's slot map is a bijection onto the tile (every element copied
  exactly once);
* every fragment read finds the element it stands for;
* every global address of a full stage, a tail stage and the clamped rows
  stays inside the operand, and every 32-bit offset is non-negative;
* the short-reduction kernel's waits never allow a DMA still in flight
  (each wait count is at most the operations really issued after it) and
  fit the 6-bit counter.

A change to a slot map, a tile shape or a launcher's shape choice that
breaks any of these fails here, on the CPU, before it reaches a GPU.
"""
import itertools

import pytest

SBK = 32  # reduction entries per stage


# ------------------------------------------------------------ operand types
class SKc:
    """k-contiguous float32 rows: element (r, k) at p[r * ld + k]."""

    def __init__(self, vec, ld, rows):
        self.vec, self.ld, self.rows = vec, ld, rows
        self.unit = 16 if vec else 4
        self.esize = 4

    def slots(self, BR):
        return BR * SBK * 4 // self.unit

    def rk(self, s):
        """(row, first k) the slot copies, within the tile and stage."""
        if self.vec:
            r = s >> 3
            return r, ((s & 7) ^ (r & 7)) << 2
        r = s >> 5
        return r, ((((s >> 2) & 7) ^ (r & 7)) << 2) | (s & 3)

    def k_of(self, s):
        return self.rk(s)[1]

    def lane_off(self, s, r0):
        r, k = self.rk(s)
        gr = r0 + r if r0 + r < self.rows else self.rows - 1
        return ((gr - r0) * self.ld + k) * 4

    def base(self, r0, k0):
        return (r0 * self.ld + k0) * 4

    def frag(self, BR, rg, q16, g4):
        """(LDS float index, (row, k)) of the 8 values of a bfloat16 fragment."""
        r = rg * 16 + q16
        out = []
        for half in range(2):
            pos = ((2 * g4 + half) ^ (r & 7)) << 2
            out += [(r * SBK + pos + e, (r, 8 * g4 + 4 * half + e)) for e in range(4)]
        return out

    def frag4(self, BR, rg, q16, g4, h):
        r = rg * 16 + q16
        pos = ((4 * h + g4) ^ (r & 7)) << 2
        return [(r * SBK + pos + j, (r, 16 * h + 4 * g4 + j)) for j in range(4)]


class SRc:
    """Row-contiguous float32 (k-major): element (r, k) at p[k * ld + r];
    row `ones` reads as 1 (set in registers).  A stage is stored in windows
    of 16 rows of one k; window (k, rg) at index 4 ((4 h + j) NG + rg) + c(k)
    with k = 16 h + 4 q + j and c(k) = (bit2 xor bit3) + 2 (bit3 xor bit4)."""

    def __init__(self, vec, ld, rows, ones):
        self.vec, self.ld, self.rows, self.ones = vec, ld, rows, ones
        self.unit = 16 if vec else 4
        self.esize = 4
        self.klast = 4 if vec else 1

    def slots(self, BR):
        return BR * SBK * 4 // self.unit

    @staticmethod
    def cls(k):
        b2, b3, b4 = (k >> 2) & 1, (k >> 3) & 1, (k >> 4) & 1
        return (b2 ^ b3) + 2 * (b3 ^ b4)

    def kr(self, s, BR):
        ng = BR // 16
        w, t = (s >> 2, (s & 3) << 2) if self.vec else (s >> 4, s & 15)
        idx, c = w >> 2, w & 3
        hj, rg = divmod(idx, ng)
        h, j = hj >> 2, hj & 3
        b3 = (c >> 1) ^ h
        b2 = (c & 1) ^ b3
        k = 16 * h + 8 * b3 + 4 * b2 + j
        assert self.cls(k) == c
        return k, 16 * rg + t

    def k_of(self, s, BR):
        return self.kr(s, BR)[0]

    def clamp(self, gr):
        return gr if gr < self.rows else self.rows - self.klast

    def rbase(self, r0):
        return r0 if r0 < self.rows - self.klast else self.rows - self.klast

    def lane_off(self, s, r0, BR):
        k, r = self.kr(s, BR)
        return (k * self.ld + (self.clamp(r0 + r) - self.rbase(r0))) * 4

    def base(self, r0, k0):
        return (k0 * self.ld + self.rbase(r0)) * 4

    def lds_pos(self, s, BR):
        """LDS float indices slot s writes."""
        return [s * (self.unit // 4) + e for e in range(self.unit // 4)]

    @staticmethod
    def at(BR, h, j, c, rg, q16):
        return 64 * ((4 * h + j) * (BR // 16) + rg) + 16 * c + q16

    def frag(self, BR, rg, q16, g4):
        h, b3 = g4 >> 1, g4 & 1
        clo, chi = b3 + 2 * (b3 ^ h), (1 ^ b3) + 2 * (b3 ^ h)
        r = rg * 16 + q16
        out = [(self.at(BR, h, e, clo, rg, q16), (r, 8 * g4 + e)) for e in range(4)]
        out += [(self.at(BR, h, e, chi, rg, q16), (r, 8 * g4 + 4 + e)) for e in range(4)]
        return out

    def frag4(self, BR, rg, q16, g4, h):
        c = ((g4 & 1) ^ (g4 >> 1)) + 2 * ((g4 >> 1) ^ h)
        r = rg * 16 + q16
        return [(self.at(BR, h, j, c, rg, q16), (r, 16 * h + 4 * g4 + j)) for j in range(4)]


class SKh:
    """bfloat16 k-contiguous rows of stride ldp (a multiple of 32, zero-padded
    beyond K), or activations stored in bfloat16 (SKb: same layout)."""

    def __init__(self, ldp, rows):
        self.ld, self.rows = ldp, rows
        self.unit = 16
        self.esize = 2

    def slots(self, BR):
        return BR * SBK * 2 // 16

    def rk(self, s):
        r = s >> 2
        return r, 8 * ((s & 3) ^ ((r >> 1) & 3))

    def k_of(self, s):
        return self.rk(s)[1]

    def lane_off(self, s, r0):
        r = s >> 2
        c = (s & 3) ^ ((r >> 1) & 3)
        gr = r0 + r if r0 + r < self.rows else self.rows - 1
        return ((gr - r0) * self.ld + 8 * c) * 2

    def base(self, r0, k0):
        return (r0 * self.ld + k0) * 2

    def frag(self, BR, rg, q16, g4):
        """(LDS bf16 index, (row, k)) of the 8 values of a fragment."""
        r = rg * 16 + q16
        pos = (g4 ^ ((r >> 1) & 3)) * 8
        return [(r * SBK + pos + e, (r, 8 * g4 + e)) for e in range(8)]


class SRb:
    """bfloat16 row-contiguous (k-major) activations: a 16-byte lane copies
    8 consecutive rows of one k."""

    def __init__(self, ld, rows, ones):
        self.ld, self.rows, self.ones = ld, rows, ones
        self.unit = 16
        self.esize = 2

    def slots(self, BR):
        return BR * SBK * 2 // 16

    @staticmethod
    def rot(k):
        return 2 * ((k >> 3) & 3)

    def kc(self, s, BR):
        nc = BR // 8
        k = s // nc
        c = s - k * nc - self.rot(k)
        if c < 0:
            c += nc
        return k, c

    def k_of(self, s, BR):
        return self.kc(s, BR)[0]

    def clamp(self, gr):
        return gr if gr < self.rows else self.rows - 8

    def rbase(self, r0):
        return r0 if r0 < self.rows - 8 else self.rows - 8

    def lane_off(self, s, r0, BR):
        k, c = self.kc(s, BR)
        return (k * self.ld + (self.clamp(r0 + 8 * c) - self.rbase(r0))) * 2

    def base(self, r0, k0):
        return (k0 * self.ld + self.rbase(r0)) * 2

    def frag(self, BR, rg, q16, g4):
        nc = BR // 8
        r = rg * 16 + q16
        c, w = r >> 3, r & 7
        pc = c + 2 * g4
        if pc >= nc:
            pc -= nc
        return [((8 * g4 + e) * BR + pc * 8 + w, (r, 8 * g4 + e)) for e in range(8)]


# ------------------------------------------------------------- the checks
def written(op, BR):
    """LDS element index -> (row, k) for one full stage (rows in range)."""
    out = {}
    per = op.unit // op.esize
    for s in range(op.slots(BR)):
        if isinstance(op, (SKc, SKh)):
            r, k = op.rk(s)
            if isinstance(op, SKh):
                pos = [s * 8 + e for e in range(8)]
            else:
                pos = [s * per + e for e in range(per)]
            elems = [(r, k + e) for e in range(per)]
        elif isinstance(op, SRc):
            k, r = op.kr(s, BR)
            pos = op.lds_pos(s, BR)
            elems = [(r + e, k) for e in range(per)]
        else:  # SRb
            k, c = op.kc(s, BR)
            pos = [s * 8 + e for e in range(8)]
            elems = [(8 * c + e, k) for e in range(8)]
        for p, el in zip(pos, elems):
            assert p not in out, (type(op).__name__, BR, s, p)
            out[p] = el
    return out


def fragments(op, BR, f32):
    NG = BR // 16
    for rg, q16, g4 in itertools.product(range(NG), range(16), range(4)):
        if f32:
            for h in (0, 1):
                yield op.frag4(BR, rg, q16, g4, h)
        else:
            yield op.frag(BR, rg, q16, g4)


# operand type and tile-row count (BR) pairs the launchers instantiate:
# A side of the 128- and 64-row tiles, B side of the 144-, 96- and 48-column
# tiles, both sides of the 128 x 144 weight-gradient tile, and the 32-column
# tiles of the short-reduction kernel
LAYOUTS = [
    ("SKc16", 128), ("SKc16", 64), ("SKc16", 144), ("SKc16", 96), ("SKc16", 48), ("SKc16", 32),
    ("SKc4", 128), ("SKc4", 64),
    ("SKh", 144), ("SKh", 48), ("SKh", 128), ("SKh", 32),
    ("SRc16", 128), ("SRc16", 144), ("SRc4", 128), ("SRc4", 144),
    ("SRb", 128), ("SRb", 144),
]


def make(kind, ld=4096, rows=4096):
    return {"SKc16": lambda: SKc(True, ld, rows), "SKc4": lambda: SKc(False, ld, rows), "SKh": lambda: SKh(ld, rows),
            "SRc16": lambda: SRc(True, ld, rows, -1), "SRc4": lambda: SRc(False, ld, rows, -1),
            "SRb": lambda: SRb(ld, rows, -1)}[kind]()


@pytest.mark.parametrize("kind,BR", LAYOUTS)
def test_stage_slot_map_is_a_bijection(kind, BR):
    op = make(kind)
    w = written(op, BR)
    assert len(w) == BR * SBK
    assert set(w.values()) == {(r, k) for r in range(BR) for k in range(SBK)}


@pytest.mark.parametrize("kind,BR", LAYOUTS)
def test_fragment_reads_find_their_elements(kind, BR):
    op = make(kind)
    w = written(op, BR)
    f32_ok = kind not in ("SKh", "SRb")
    for f32 in ((False, True) if f32_ok else (False,)):
        for frag in fragments(op, BR, f32):
            for pos, want in frag:
                assert w[pos] == want, (kind, BR, f32, pos, w[pos], want)


def lane_reads(op, BR, f32):
    """Per fragment-read instruction (row group, h, element): the 64 lanes'
    LDS element indices, lane = 16 g4 + q16."""
    NG = BR // 16
    for rg in range(NG):
        for h in ((0, 1) if f32 else (None,)):
            per_lane = {}
            for q16, g4 in itertools.product(range(16), range(4)):
                f = op.frag4(BR, rg, q16, g4, h) if f32 else op.frag(BR, rg, q16, g4)
                per_lane[16 * g4 + q16] = [pos for pos, _ in f]
            for e in range(len(per_lane[0])):
                yield [per_lane[lane][e] for lane in range(64)]


# SRb on the 144-wide side (a bfloat16 operand of at most 144 rows, which no
# workload has: their bfloat16 activations are 1440 wide) rotates its last
# chunks around the k-line and conflicts two ways there; it stays correct.
@pytest.mark.parametrize("kind,BR", [(k, b) for k, b in LAYOUTS if k.startswith("SR") and (k, b) != ("SRb", 144)])
def test_element_reads_are_free_of_bank_conflicts(kind, BR):
    """The row-contiguous operands read their fragments one dword per lane
    (float32 values; bfloat16 rows read as the dword holding a row pair).
    Each read instruction is checked in two bank models: 64 banks of 4 bytes
    over all 64 lanes, and 32 banks over each half-wave (lanes 0-31, 32-63)
    -- the one the conflict counters follow for these reads.  In both, the
    lanes hit different banks or the same dword (a broadcast), for the FP32
    and the BF16 fragment alike."""
    op = make(kind)
    for f32 in ((False, True) if kind.startswith("SRc") else (False,)):
        for addrs in lane_reads(op, BR, f32):
            for banks, groups in ((64, (range(64),)), (32, (range(32), range(32, 64)))):
                for lanes in groups:
                    dword = {}
                    for lane in lanes:
                        d = addrs[lane] * op.esize // 4
                        assert dword.setdefault(d % banks, d) == d, (kind, BR, f32, banks, lane)


@pytest.mark.parametrize("kind", ["SKc16", "SKc4", "SKh"])
def test_tail_stage_copies_exactly_the_range(kind):
    """In the stage where the reduction ends (krem < 32 entries left), the
    slots whose entries lie at or beyond the end copy zeros; the others
    copy exactly the entries inside the range (16-byte lanes need kend % 4
    == 0 for float32, % 8 for bfloat16, so a lane is wholly in or out)."""
    op = make(kind)
    per = op.unit // op.esize
    step = 4 if kind == "SKc16" else (8 if kind == "SKh" else 1)
    for krem in range(step, SBK, step):
        for s in range(op.slots(128)):
            k = op.k_of(s)
            inside = k < krem
            assert inside == (k + per - 1 < krem)


# ---------------------------------------------- workload operand shapes
def pad32(x):
    return (x + 31) // 32 * 32


# (C, O, K_in, K_out) of every folded layer in the workloads and tests:
# three-shell stack 3->32->3 (order 8), four-layer net 3->32->64->32->3,
# learned predictor 3->64 (order 4 -> 8) ->64->3, one-shell 1->8 (order 4),
# and the test shapes 3->5 (4 -> 8), 5->16 / 16->5 (order 6), 16 (order 2)
LAYERS = sorted({
    (3, 32, 45, 45), (32, 3, 45, 45), (32, 64, 45, 45), (64, 32, 45, 45),
    (3, 64, 15, 45), (64, 64, 45, 45), (64, 3, 45, 45), (1, 8, 15, 15),
    (3, 5, 15, 45), (5, 16, 28, 28), (16, 5, 28, 28), (3, 16, 6, 6), (16, 3, 6, 6),
})
VOXELS = [1, 33, 203, 8192, 1 << 20]


def tile_starts(total, BR):
    n = (total + BR - 1) // BR
    idx = list(range(n)) if n <= 6 else [0, 1, n - 3, n - 2, n - 1]
    return [i * BR for i in idx]


def stage_starts(kend):
    n = (kend + SBK - 1) // SBK
    idx = list(range(n)) if n <= 4 else [0, 1, n - 2, n - 1]
    return [i * SBK for i in idx]


def check_k_contiguous(op, BR, M, kend, alloc_bytes, table=False):
    """Every address a stage of a k-contiguous operand copies is inside it.
    A table (zero-padded rows) is copied whole, also in the last stage."""
    for r0 in tile_starts(M, BR):
        for k0 in stage_starts(kend):
            krem = kend - k0
            for s in range(op.slots(BR)):
                o = op.lane_off(s, r0)
                assert 0 <= o < 2 ** 32
                if not table and krem < SBK and op.k_of(s) >= krem:
                    continue  # copies zeros
                a = op.base(r0, k0) + o
                assert 0 <= a and a + op.unit <= alloc_bytes, (r0, k0, s, a, alloc_bytes)


def check_row_contiguous(op, BR, rows, kbeg, kend, alloc_bytes):
    for r0 in tile_starts(rows + (1 if op.ones >= 0 else 0), BR):
        for k0 in [kbeg + s for s in stage_starts(kend - kbeg)]:
            krem = kend - k0
            for s in range(op.slots(BR)):
                o = op.lane_off(s, r0, BR)
                assert 0 <= o < 2 ** 32, (r0, s, o)
                if krem < SBK and op.k_of(s, BR) >= krem:
                    continue
                a = op.base(r0, k0) + o
                assert 0 <= a and a + op.unit <= alloc_bytes, (r0, k0, s, a, alloc_bytes)


def tiled_cfg(N, f32):
    """(BM, BN) the tiled core launches for a table GEMM with N columns."""
    if N <= 96:
        return 128, 48
    if f32 and N > 144:
        return 64, 96
    return 128, 144


@pytest.mark.parametrize("layer", LAYERS)
@pytest.mark.parametrize("V", VOXELS)
def test_table_gemm_addresses_stay_inside_their_operands(layer, V):
    """Forward (A = layer input [V][C K_in], table [O K_out][pad32(C K_in)])
    and input gradient (A = output gradient [V][O K_out], table
    [C K_in][pad32(O K_out)]), float32 or bfloat16 activations and both
    precisions' tables, for the tile shape the launcher picks."""
    C, O, Ki, Ko = layer
    for K, N in ((C * Ki, O * Ko), (O * Ko, C * Ki)):
        for f32 in (True, False):
            BM, BN = tiled_cfg(N, f32)
            A = [SKc(K % 4 == 0, K, V)] + ([SKc(False, K, V)] if K % 4 == 0 else [])
            for a in A:
                check_k_contiguous(a, BM, V, K, V * K * 4)
            if not f32 and K % 8 == 0:  # activations stored in bfloat16
                check_k_contiguous(SKh(K, V), BM, V, K, V * K * 2)
            ldb = pad32(K)
            tab = SKc(True, ldb, N) if f32 else SKh(ldb, N)
            check_k_contiguous(tab, BN, N, K, N * ldb * tab.esize, table=True)
            if astat_ok(K, N):  # the short-reduction kernel: 32-column tiles
                check_k_contiguous(SKc(True, ldb, N) if f32 else SKh(ldb, N), 32, N, K, N * ldb * tab.esize,
                                   table=True)


def grad_splits(V, M, N1):
    def split_len(Kv, s):
        ks = (Kv + s - 1) // s
        return (ks + 31) // 32 * 32
    big, small = max(M, N1), min(M, N1)
    tiles = (big + 127) // 128 if small <= 144 else ((big + 63) // 64) * ((small + 63) // 64)
    s = min(128, max(1, (2048 + tiles - 1) // tiles))
    s = min(s, max(1, V // 512))
    while s > 1 and (V + split_len(V, s) - 1) // split_len(V, s) != s:
        s -= 1
    return s, split_len(V, s)


@pytest.mark.parametrize("layer", LAYERS)
@pytest.mark.parametrize("V", VOXELS)
def test_weight_gradient_addresses_stay_inside_their_operands(layer, V):
    """dT = sum_v g[v][m] act[v][n] with a ones column at n = C K_in: both
    operands row-contiguous (k = voxel), split over voxel slices; the tile
    that starts at or past the ones row uses the clamped tile start (its
    32-bit offsets would otherwise be negative)."""
    C, O, Ki, Ko = layer
    M, CK = O * Ko, C * Ki
    N1 = CK + 1
    splits, ks = grad_splits(V, M, N1)
    assert (V + ks - 1) // ks == splits and ks % SBK == 0
    for z in [0, splits - 1]:
        kbeg, kend = z * ks, min(V, z * ks + ks)
        ops = []
        g_ops = [SRc(M % 4 == 0, M, M, -1)] + ([SRb(M, M, -1)] if M % 8 == 0 else [])
        a_ops = [SRc(CK % 4 == 0, CK, CK, CK)] + ([SRb(CK, CK, CK)] if CK % 8 == 0 else [])
        for g in g_ops:
            ops.append((g, M, V * M * g.esize))
        for a in a_ops:
            ops.append((a, CK, V * CK * a.esize))
        for op, rows, alloc in ops:
            for br in (128, 144):  # either side of the 128 x 144 tile
                if isinstance(op, SRb) and rows % 8:
                    continue
                check_row_contiguous(op, br, rows, kbeg, kend, alloc)


# ------------------------------------------------ short-reduction kernel
KS = 5


def astat_ok(K, N):
    return 128 < K <= 160 and N % 32 == 0 and N <= 1440


def astat_dma(op, BN, wave):
    """(LDS byte offset in the tile, global byte offset from the tile's first
    table row) of every lane copy of the wave's instructions."""
    NI = op.slots(BN) // 64
    NIT = KS * NI
    KB = op.esize
    out = []
    for k in range((NIT + 3) // 4):
        q = wave + 4 * k
        if q >= NIT:
            continue
        sl, ins = q // NI, q % NI
        slab = BN * SBK * op.esize
        for lane in range(64):
            s = ins * 64 + lane
            out.append((sl * slab + ins * 64 * 16 + lane * 16, op.lane_off(s, 0) + sl * SBK * KB, sl, s))
    return out


@pytest.mark.parametrize("f32", [True, False])
def test_short_reduction_dma_covers_each_tile_once(f32):
    BN, ldb, N = 32, 160, 1440
    op = SKc(True, ldb, N) if f32 else SKh(ldb, N)
    tile_bytes = KS * BN * SBK * op.esize
    seen = {}
    for wave in range(4):
        for lds, glob, sl, s in astat_dma(op, BN, wave):
            assert lds not in seen
            seen[lds] = (sl, s)
            assert 0 <= glob < 2 ** 32
            # the slice's element the slot copies, in the layout frag reads
            r, k = op.rk(s)
            assert glob == (r * ldb + SBK * sl + k) * op.esize
    assert sorted(seen) == list(range(0, tile_bytes, 16))
    # the last tile's copies stay inside the table
    last = (N // BN - 1) * BN * ldb * op.esize
    top = max(g for w in range(4) for _, g, _, _ in astat_dma(op, BN, w))
    assert last + top + 16 <= N * ldb * op.esize


@pytest.mark.parametrize("f32,D", [(True, 1), (False, 3), (False, 2)])
@pytest.mark.parametrize("N", [1440, 448, 96, 32])
def test_short_reduction_waits_never_cover_a_dma_in_flight(f32, D, N):
    """Replays the issue order of one wave (prologue DMA of tiles 0..D-1;
    then per tile t: wait, DMA of tile t+D, MFMAs, stores) and checks that
    each wait's vmcnt immediate is at most the number of vector-memory
    operations really issued after the DMA of the tile it waits for, in a
    block whose rows are all below M (elsewhere the waits count no stores)."""
    BN, TM = 32, 2
    TN = BN // 16
    op = SKc(True, 160, N) if f32 else SKh(160, N)
    NI = op.slots(BN) // 64
    NIT = KS * NI
    IW = NIT // 4
    half = not f32
    SW = TM * ((TN + 1) // 2 if half else TN)  # the kernel's lower bound
    assert D * SW + (D - 1) * IW < 64
    NT = N // BN
    for wave in range(4):
        nq = (NIT - wave + 3) // 4
        # stores per tile: the data stores (ReLU bits go to LDS, and to
        # memory once after the loop)
        stores = TM * ((TN // 2) + (TN % 2) if half else TN)
        log = []  # ("dma", t) or ("st", t), in issue order
        for t in range(min(D, NT)):
            log += [("dma", t)] * nq
        for t in range(NT):
            if t >= D:
                later = min(D - 1, NT - 1 - t)
                imm = D * SW + later * IW
                last = max(i for i, e in enumerate(log) if e == ("dma", t))
                assert imm <= len(log) - 1 - last, (wave, t, imm)
            if t + D < NT:
                log += [("dma", t + D)] * nq
            log += [("st", t)] * stores
