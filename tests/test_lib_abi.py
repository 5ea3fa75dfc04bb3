"""Host-side checks of libqva (no GPU needed, nothing is launched).

* the library loads and exports every function include/qva.h declares;
* argument validation returns the documented status before any launch;
* the pass planner covers every qubit once per layer, orders phases between
  layers, and has the documented pass count p(P-1)+1.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qva.h")

_lib = pytest.importorskip("paper_2110_03963_amd._lib")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2110_03963_amd import build
        build.build()
    return _lib.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qva_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_status_strings(lib):
    for st in [0, -1, -2, -3, -4, -5, -6, -7]:
        assert lib.qva_status_string(st)
    assert lib.qva_status_string(-4) == b"workspace missing or too small"
    assert b"gfx950" in lib.qva_version()


FAKE = 0x7F0000001000  # never dereferenced: every call below fails validation first


def _prob(mixer=0, n=20, q=FAKE, lam=None, kind=0, n_states=0, terms=None, n_terms=0):
    return _lib.QvaProblem(mixer, n, q, lam, kind, n_states, terms, n_terms)


def test_validation_errors(lib):
    S = _lib
    assert lib.qva_init_uniform(None, 16, None) == S.QVA_ERR_ARG
    assert lib.qva_init_uniform(FAKE, 0, None) == S.QVA_ERR_SIZE
    assert lib.qva_init_uniform(FAKE + 8, 16, None) == S.QVA_ERR_ALIGN
    assert lib.qva_phase(FAKE, None, 16, 0.1, None) == S.QVA_ERR_ARG
    assert lib.qva_phase(FAKE, FAKE + 4, 16, 0.1, None) == S.QVA_ERR_ALIGN
    assert lib.qva_mix_x(FAKE, 0, 0.1, None) == S.QVA_ERR_SIZE
    assert lib.qva_mix_x(FAKE, 34, 0.1, None) == S.QVA_ERR_SIZE
    assert lib.qva_mix_x(FAKE + 8, 5, 0.1, None) == S.QVA_ERR_ALIGN
    assert lib.qva_mix_x(None, 5, 0.1, None) == S.QVA_ERR_ARG
    assert lib.qva_expectation(FAKE, FAKE, 1 << 20, FAKE, None, None, 0, None) == S.QVA_ERR_WORKSPACE
    assert lib.qva_expectation(FAKE, FAKE, 0, FAKE, None, FAKE, 1 << 20, None) == S.QVA_ERR_SIZE


def test_evolve_validation(lib):
    S = _lib
    pr = _prob(n=20)
    ref = ctypes.byref
    ws = lib.qva_workspace_bytes(ref(pr), 3, 0)
    assert ws == 16 * (1 << 8)
    # workspace too small / missing
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, 3, FAKE, FAKE, None, 0, FAKE, ws - 16, None) == S.QVA_ERR_WORKSPACE
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, 3, FAKE, FAKE, None, 0, None, 0, None) == S.QVA_ERR_WORKSPACE
    # bad depth, bad flags, null parameters, misaligned outputs
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, -1, FAKE, FAKE, None, 0, FAKE, ws, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, 3, FAKE, FAKE, None, 4, FAKE, ws, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve(ref(pr), None, FAKE, 3, FAKE, FAKE, None, 0, FAKE, ws, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, 3, FAKE, FAKE + 4, None, 0, FAKE, ws, None) == S.QVA_ERR_ALIGN
    assert lib.qva_evolve(ref(pr), FAKE, FAKE, 3, FAKE + 8, FAKE, None, 0, FAKE, ws, None) == S.QVA_ERR_ALIGN
    # problem descriptor errors
    for bad, st in [(_prob(n=0), S.QVA_ERR_SIZE), (_prob(n=34), S.QVA_ERR_SIZE),
                    (_prob(mixer=7), S.QVA_ERR_ARG), (_prob(q=None), S.QVA_ERR_ARG),
                    (_prob(q=FAKE + 2), S.QVA_ERR_ALIGN),
                    (_prob(mixer=1, kind=0, lam=None), S.QVA_ERR_ARG),
                    (_prob(mixer=1, kind=9, lam=FAKE), S.QVA_ERR_ARG)]:
        assert lib.qva_evolve(ref(bad), FAKE, FAKE, 3, FAKE, FAKE, None, 0, FAKE, 1 << 30, None) == st
    assert lib.qva_evolve(None, FAKE, FAKE, 3, FAKE, FAKE, None, 0, FAKE, 1 << 30, None) == S.QVA_ERR_ARG
    assert lib.qva_workspace_bytes(None, 3, 0) == 0


def _plan(lib, n, p, flags=0):
    pr = _prob(n=n)
    cnt = lib.qva_plan(ctypes.byref(pr), p, 0, flags, None, 0)
    assert cnt > 0
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, 0, flags, arr, cnt) == cnt
    return list(arr)


@pytest.mark.parametrize("n", [13, 20, 21, 22, 26, 28, 30, 33])
@pytest.mark.parametrize("p", [1, 2, 3, 8, 12])
def test_plan_schedule(lib, n, p):
    plan = _plan(lib, n, p)
    assert plan[-1].kind == 8  # final reduce
    passes = plan[:-1]
    groups = sorted({(x.group_first, x.group_bits) for x in passes})
    # groups tile the qubits [0, n) exactly
    covered = []
    for k, b in groups:
        covered.extend(range(k, k + b))
    assert covered == list(range(n))
    P = len(groups)
    assert len(passes) == p * (P - 1) + 1
    # replay: each layer applies every group once, phase k between layers k-1 and k
    done = {L: set() for L in range(p)}
    phased = set()
    for x in passes:
        if x.phase_layer >= 0 and x.kind == 1:
            assert x.phase_layer == 0
            phased.add(0)
        if x.mix_layer >= 0:
            L = x.mix_layer
            assert L in phased
            assert (x.group_first, x.group_bits) not in done[L]
            done[L].add((x.group_first, x.group_bits))
        if x.kind == 3:
            L2 = x.phase_layer
            assert L2 == x.mix_layer + 1 == x.mix_layer2
            assert len(done[L2 - 1]) == P, "phase before the previous layer finished"
            phased.add(L2)
            done[L2].add((x.group_first, x.group_bits))
    for L in range(p):
        assert len(done[L]) == P
    assert passes[0].kind == 1 and passes[-1].kind in (4, 5)
    # high groups keep >= 8 contiguous amplitudes (128 bytes) per row
    for x in passes:
        if x.group_first > 0:
            assert x.col_bits >= 3 and x.col_bits + x.group_bits == 12


def test_plan_bytes(lib):
    N = 1 << 28
    plan = _plan(lib, 28, 8, flags=1)
    total = sum(x.bytes for x in plan[:-1])
    # 1 first (24 B/amp) + 8 middle (32) + 7 boundary (40) + 1 last (24)
    assert total == N * (24 + 8 * 32 + 7 * 40 + 24)
    plan = _plan(lib, 28, 8, flags=0)
    assert plan[-2].kind == 5 and plan[-2].bytes == 40 * N


def test_plan_small_and_depth_zero(lib):
    plan = _plan(lib, 10, 4)
    assert [x.kind for x in plan] == [0]
    plan = _plan(lib, 20, 0)
    assert [x.kind for x in plan] == [6, 7, 8]


@pytest.mark.parametrize("n", [13, 20, 26, 33])
@pytest.mark.parametrize("p", [1, 2, 6])
def test_plan_complete_closed_form(lib, n, p):
    """Complete graph (lambda kind 2), n > 12: one streaming pass per layer
    plus a reduction of the state sum after every pass that writes."""
    pr = _prob(mixer=1, n=n, kind=2, lam=None)
    N = 1 << n
    for flags, last in [(1, 28), (0, 29)]:
        cnt = lib.qva_plan(ctypes.byref(pr), p, 0, flags, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        assert lib.qva_plan(ctypes.byref(pr), p, 0, flags, arr, cnt) == cnt
        kinds = [x.kind for x in arr]
        assert kinds == [26, 30] + [27, 30] * (p - 1) + [last, 8]
        layers = [(x.mix_layer, x.phase_layer) for x in arr if x.kind in (26, 27, 28, 29)]
        assert layers == [(-1, 0)] + [(k, k + 1) for k in range(p - 1)] + [(p - 1, -1)]
        parts = 16 * (N >> 12)
        bytes_ = [x.bytes for x in arr if x.kind in (26, 27, 28, 29)]
        assert bytes_ == [24 * N + parts] + [40 * N + parts] * (p - 1) + [(24 if flags else 40) * N + parts]
    # the running state sum takes 256 bytes after the (256-aligned) partials
    assert lib.qva_workspace_bytes(ctypes.byref(pr), p, 0) == ((16 * (N >> 12) + 255) // 256) * 256 + 256
    # depth 0 and small n keep their plans
    assert [x for x in [lib.qva_plan(ctypes.byref(pr), 0, 0, 0, None, 0)]] == [3]
    small = _prob(mixer=1, n=12, kind=2, lam=None)
    assert lib.qva_plan(ctypes.byref(small), p, 0, 0, None, 0) == 1


@pytest.mark.parametrize("n", [13, 26])
@pytest.mark.parametrize("p", [1, 3, 6])
def test_grad_plan_complete_closed_form(lib, n, p):
    """qva_grad with the complete graph: forward without the last mixer, the
    turn, one backward pass per layer, each followed by its fixed-order sums."""
    pr = _prob(mixer=1, n=n, kind=2, lam=None)
    cnt = lib.qva_plan(ctypes.byref(pr), p, 1, 0, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, 1, 0, arr, cnt) == cnt
    kinds = [x.kind for x in arr]
    assert kinds == ([26, 30] + [27, 30] * (p - 1) + [31, 33] + [32, 33] * p + [8, 25])
    back = [(x.mix_layer, x.phase_layer) for x in arr if x.kind == 32]
    assert back == [(k, k) for k in range(p - 1, -1, -1)]
    N = 1 << n
    bytes_ = [x.bytes for x in arr if x.kind in (31, 32)]
    parts = 64 * (N >> 12)
    assert bytes_[0] == 56 * N + 16 * 5 * (N >> 12)
    assert bytes_[1:] == [72 * N + parts] * (p - 1) + [40 * N + parts]
    # workspace: (f, norm) partials, 8 doubles per block, running sums, 2p sums
    ws = lib.qva_workspace_bytes(ctypes.byref(pr), p, 1)
    assert ws >= 16 * (N >> 12) + 64 * (N >> 12) + 64 + 16 * p


def test_n_states_validation(lib):
    """A non-power-of-two N must satisfy 2^(n-1) < N < 2^n and is accepted
    for the complete-graph mixer only."""
    S = _lib
    ref = ctypes.byref
    ws = 1 << 30
    ok = _prob(mixer=1, n=17, kind=2, n_states=100003)
    assert lib.qva_plan(ref(ok), 3, 0, 0, None, 0) > 0
    for bad, st in [(_prob(mixer=1, n=17, kind=2, n_states=65536), S.QVA_ERR_SIZE),
                    (_prob(mixer=1, n=17, kind=2, n_states=131073), S.QVA_ERR_SIZE),
                    (_prob(mixer=1, n=17, kind=2, n_states=-5), S.QVA_ERR_SIZE),
                    (_prob(mixer=1, n=32, kind=1, n_states=(1 << 31) + 5), S.QVA_ERR_UNSUPPORTED),
                    (_prob(mixer=0, n=17, n_states=100003), S.QVA_ERR_UNSUPPORTED)]:
        assert lib.qva_evolve(ref(bad), FAKE, FAKE, 3, FAKE, FAKE, None, 0, FAKE, ws, None) == st
        assert lib.qva_plan(ref(bad), 3, 0, 0, None, 0) == st
    # n_states equal to 2^n is the same as 0
    same = _prob(mixer=1, n=17, kind=2, n_states=1 << 17)
    assert lib.qva_workspace_bytes(ref(same), 3, 0) == lib.qva_workspace_bytes(ref(_prob(mixer=1, n=17, kind=2)), 3, 0)


@pytest.mark.parametrize("N,n", [(3, 2), (1000, 10), (4097, 13), (100003, 17), (5000011, 23)])
@pytest.mark.parametrize("p", [0, 1, 4])
def test_plan_complete_any_n(lib, N, n, p):
    """Closed-form plans for a non-power-of-two N (the solution count of a
    constrained problem): one pass per layer, ceil(N / 4096) blocks."""
    pr = _prob(mixer=1, n=n, kind=2, n_states=N)
    blocks = -(-N // 4096)
    parts = 16 * blocks
    cnt = lib.qva_plan(ctypes.byref(pr), p, 0, 1, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, 0, 1, arr, cnt) == cnt
    kinds = [x.kind for x in arr]
    if p == 0:
        assert kinds == [6, 7, 8]
    else:
        assert kinds == [26, 30] + [27, 30] * (p - 1) + [28, 8]
        b = [x.bytes for x in arr if x.kind in (26, 27, 28)]
        assert b == [24 * N + parts] + [40 * N + parts] * (p - 1) + [24 * N + parts]
    expect_parts = min(-(-N // 4096), 4096)
    ws = lib.qva_workspace_bytes(ctypes.byref(pr), p, 0)
    assert ws == ((16 * max(blocks, expect_parts) + 255) // 256) * 256 + 256
    if p > 0:
        cnt = lib.qva_plan(ctypes.byref(pr), p, 1, 0, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        assert lib.qva_plan(ctypes.byref(pr), p, 1, 0, arr, cnt) == cnt
        assert [x.kind for x in arr] == [26, 30] + [27, 30] * (p - 1) + [31, 33] + [32, 33] * p + [8, 25]
        assert lib.qva_workspace_bytes(ctypes.byref(pr), p, 1) > 0


@pytest.mark.parametrize("N,n", [(1009, 10), (4097, 13), (100003, 17), (3000017, 22)])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p", [1, 3])
def test_plan_bluestein(lib, N, n, kind, p):
    """Ring / array circulant over N (not a power of two): two filter spectra,
    psi_0, then per layer two convolutions over the padded M >= 2N - 1."""
    pr = _prob(mixer=1, n=n, kind=kind, lam=FAKE if kind == 0 else None, n_states=N)
    M = 1 << max(13, (2 * N - 2).bit_length())
    for flags, last in [(1, 40), (0, 41)]:
        cnt = lib.qva_plan(ctypes.byref(pr), p, 0, flags, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        assert lib.qva_plan(ctypes.byref(pr), p, 0, flags, arr, cnt) == cnt
        kinds = [x.kind for x in arr]
        mids = sorted({x.group_first for x in arr if x.kind == 10})
        nm = len(mids)
        conv = [10] * nm
        back = [12] * nm
        layer = conv + [37] + back + [38] + conv + [37] + back
        expect = [51] + ([34] + conv + [35]) * 2 + [36]  # 51: the low-group root table
        for k in range(p):
            expect += layer + ([39] if k + 1 < p else [last])
        assert kinds == expect + [8]
        # the groups tile the padded index bits
        bits = sorted({(x.group_first, x.group_bits) for x in arr if x.group_first >= 0})
        covered = []
        for k0, b in bits:
            covered.extend(range(k0, k0 + b))
        assert covered == list(range(M.bit_length() - 1))
        mul = [x.bytes for x in arr if x.kind == 37]
        assert mul == [48 * M] * (2 * p)
    assert lib.qva_workspace_bytes(ctypes.byref(pr), p, 0) >= 3 * 16 * M
    # the adjoint: the filters and the forward up to its last convolution, the
    # turn, then per layer backwards two convolutions per vector around the
    # lambda pass, and the phase pass (the final one for layer 0)
    cnt = lib.qva_plan(ctypes.byref(pr), p, 1, 0, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, 1, 0, arr, cnt) == cnt
    kinds = [x.kind for x in arr]
    mids = sorted({x.group_first for x in arr if x.kind == 10})
    conv = [10] * len(mids)
    back = [12] * len(mids)
    fwd = [51] + ([34] + conv + [35]) * 2 + [36]
    for k in range(p):
        fwd += conv + [37] + back + [38] + conv + [37] + back + ([39] if k + 1 < p else [])
    walk = []
    for k in range(p - 1, -1, -1):
        walk += (conv + [37] + back) * 2 + [47] + (conv + [37] + back) * 2 + [48 if k > 0 else 49]
    assert kinds == fwd + [46] + walk + [8, 25]
    assert [x.mix_layer for x in arr if x.kind == 47] == list(range(p - 1, -1, -1))
    assert [x.phase_layer for x in arr if x.kind in (48, 49)] == list(range(p - 1, -1, -1))
    assert lib.qva_workspace_bytes(ctypes.byref(pr), p, 1) >= 4 * 16 * M + 2 * p * 8 * (M >> 12)


def _grad_plan(lib, mixer, n, p, kind=1):
    pr = _prob(mixer=mixer, n=n, lam=FAKE if kind == 0 else None, kind=kind)
    cnt = lib.qva_plan(ctypes.byref(pr), p, 1, 0, None, 0)
    assert cnt > 0
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, 1, 0, arr, cnt) == cnt
    return list(arr)


@pytest.mark.parametrize("n", [13, 21, 22, 28, 30])
@pytest.mark.parametrize("p", [1, 2, 5, 12])
def test_grad_plan_hypercube(lib, n, p):
    """Every (layer, qubit group) rotation of the forward is undone by exactly
    one backward pass, and every phase by exactly one."""
    plan = _grad_plan(lib, 0, n, p)
    kinds = [x.kind for x in plan]
    assert kinds[-2:] == [8, 25]
    assert kinds.count(18) == 1 and kinds.count(21) == 1
    back = plan[kinds.index(18):-2]
    fwd = plan[:kinds.index(18)]
    assert all(x.kind in (1, 2, 3) for x in fwd)
    undone = []
    phases = []
    for x in back:
        g = (x.group_first, x.group_bits)
        if x.kind in (18, 19):
            undone.append((x.mix_layer, g))
        elif x.kind == 20:
            undone += [(x.mix_layer, g), (x.mix_layer2, g)]
            phases.append(x.phase_layer)
            assert x.mix_layer == x.phase_layer == x.mix_layer2 + 1
        elif x.kind == 21:
            undone.append((0, g))
            phases.append(0)
    groups = {(x.group_first, x.group_bits) for x in plan if x.group_first >= 0}
    assert sorted(undone) == sorted((L, g) for L in range(p) for g in groups)
    assert sorted(phases) == list(range(p))
    # backward layers are visited from the last layer down
    layers = [x.mix_layer for x in back]
    assert layers == sorted(layers, reverse=True)


@pytest.mark.parametrize("n", [13, 22, 26])
@pytest.mark.parametrize("p", [1, 3, 6])
def test_grad_plan_circulant(lib, n, p):
    plan = _grad_plan(lib, 1, n, p, kind=1)
    kinds = [x.kind for x in plan]
    back = plan[kinds.index(18):-2]
    assert sorted(x.mix_layer for x in back if x.kind == 24) == list(range(p))
    assert sorted(x.phase_layer for x in back if x.kind in (20, 21)) == list(range(p))
    # forward DIF passes are undone by DIT passes and vice versa
    fwd = plan[:kinds.index(18)]
    assert sum(x.kind == 10 for x in fwd) == sum(x.kind == 23 for x in back)
    assert sum(x.kind == 12 for x in fwd) == sum(x.kind == 22 for x in back)


def _batch_items(specs):
    arr = (_lib.QvaBatchItem * len(specs))()
    for i, (n, p) in enumerate(specs):
        arr[i] = _lib.QvaBatchItem(n, p, FAKE, FAKE, FAKE, FAKE, FAKE + 4096, FAKE, FAKE, FAKE)
    return arr


@pytest.mark.parametrize("align", [0, 1, 2])
def test_batch_plan_counts(lib, align):
    """Host-side batch plan: every tile of every pass appears once; rounds are
    the deepest instance's pass count; n = 12 instances are single items."""
    specs = [(12, 3), (13, 1), (14, 2), (17, 5), (21, 8), (22, 4), (12, 1)]
    arr = _batch_items(specs)
    plan = ctypes.c_void_p()
    assert lib.qva_batch_create(arr, len(specs), align, ctypes.byref(plan)) == 0
    try:
        def npass(n, p):
            if n == 12:
                return 1
            P = 2 if n <= 21 else 3
            m = p * (P - 1) + 1  # forward passes of the evolution
            return 2 * m  # m - 1 forward, the turnaround, m - 1 backward, the reduce

        def tiles(n, p):
            if n == 12:
                return 1
            P = 2 if n <= 21 else 3
            m = p * (P - 1) + 1
            return (2 * m - 1) * (1 << (n - 12)) + 1

        assert lib.qva_batch_rounds(plan) == max(npass(n, p) for n, p in specs)
        assert lib.qva_batch_tiles(plan) == sum(tiles(n, p) for n, p in specs)
        assert lib.qva_batch_launches(plan) >= lib.qva_batch_rounds(plan)
        assert lib.qva_batch_workspace_bytes(plan) > 0
    finally:
        lib.qva_batch_destroy(plan)


def test_batch_validation(lib):
    plan = ctypes.c_void_p()
    for specs, st in [([(11, 2)], _lib.QVA_ERR_SIZE), ([(31, 2)], _lib.QVA_ERR_SIZE),
                      ([(14, 0)], _lib.QVA_ERR_SIZE), ([(14, 65)], _lib.QVA_ERR_SIZE)]:
        assert lib.qva_batch_create(_batch_items(specs), 1, 0, ctypes.byref(plan)) == st
    arr = _batch_items([(14, 2)])
    arr[0].psi = arr[0].chi
    assert lib.qva_batch_create(arr, 1, 0, ctypes.byref(plan)) == _lib.QVA_ERR_ARG
    arr = _batch_items([(14, 2)])
    arr[0].psi = FAKE + 8
    assert lib.qva_batch_create(arr, 1, 0, ctypes.byref(plan)) == _lib.QVA_ERR_ALIGN
    assert lib.qva_batch_create(_batch_items([(14, 2)]), 1, 7, ctypes.byref(plan)) == _lib.QVA_ERR_ARG
    assert lib.qva_batch_create(_batch_items([(14, 2)]), 0, 0, ctypes.byref(plan)) == _lib.QVA_ERR_ARG
    for lanes in (0, _lib.QVA_BATCH_MAX_LANES + 1, -1):
        assert lib.qva_batch_create_lanes(_batch_items([(14, 2)]), 1, 0, lanes,
                                          ctypes.byref(plan)) == _lib.QVA_ERR_ARG


@pytest.mark.parametrize("lanes", [1, 2, 3, 8])
@pytest.mark.parametrize("align", [0, 1, 2])
def test_batch_plan_lanes(lib, lanes, align):
    """Lanes split the instances into independent sequences of rounds: every
    tile still appears once, no lane needs more rounds than the deepest
    instance, each launch belongs to one round, and with one lane the plan is
    qva_batch_create's."""
    specs = [(12, 3), (13, 1), (14, 2), (17, 5), (21, 8), (22, 4), (12, 1), (16, 6), (18, 2)]
    arr = _batch_items(specs)
    one, plan = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.qva_batch_create(arr, len(specs), align, ctypes.byref(one)) == 0
    assert lib.qva_batch_create_lanes(arr, len(specs), align, lanes, ctypes.byref(plan)) == 0
    try:
        assert lib.qva_batch_tiles(plan) == lib.qva_batch_tiles(one)
        assert lib.qva_batch_rounds(plan) <= lib.qva_batch_rounds(one)
        assert lib.qva_batch_launches(plan) >= lib.qva_batch_launches(one)
        rounds = ctypes.c_int()
        wgs = ctypes.c_int64()
        total = 0
        last = -1
        for i in range(lib.qva_batch_launches(plan)):
            assert lib.qva_batch_launch_info(plan, i, ctypes.byref(rounds), ctypes.byref(wgs), None) == 0
            assert rounds.value >= last  # launches in round order
            last = rounds.value
            total += wgs.value
        assert total == lib.qva_batch_tiles(plan)
        if lanes == 1:
            assert lib.qva_batch_launches(plan) == lib.qva_batch_launches(one)
            assert lib.qva_batch_workspace_bytes(plan) == lib.qva_batch_workspace_bytes(one)
    finally:
        lib.qva_batch_destroy(plan)
        lib.qva_batch_destroy(one)


# ------------------------------------------------------------ extended QAOA
def test_zterm_validation(lib):
    """Z-string terms: hypercube mixer only, 1..QVA_MAX_TERMS, non-null and
    8-byte aligned; checked before anything is launched."""
    S = _lib
    assert S.QVA_MAX_TERMS == 1024
    ok = _prob(n=20, terms=FAKE, n_terms=5)
    assert lib.qva_plan(ctypes.byref(ok), 2, 0, 0, None, 0) > 0
    assert lib.qva_plan(ctypes.byref(ok), 2, 1, 0, None, 0) > 0
    for bad, st in [(_prob(n=20, terms=None, n_terms=5), S.QVA_ERR_ARG),
                    (_prob(n=20, terms=FAKE, n_terms=-1), S.QVA_ERR_ARG),
                    (_prob(n=20, terms=FAKE, n_terms=1025), S.QVA_ERR_ARG),
                    (_prob(n=20, terms=FAKE + 4, n_terms=3), S.QVA_ERR_ALIGN),
                    (_prob(mixer=1, n=20, kind=1, terms=FAKE, n_terms=3), S.QVA_ERR_UNSUPPORTED)]:
        assert lib.qva_plan(ctypes.byref(bad), 2, 0, 0, None, 0) == st
        assert lib.qva_workspace_bytes(ctypes.byref(bad), 2, 1) == 0
        assert lib.qva_evolve(ctypes.byref(bad), FAKE, FAKE, 2, FAKE, FAKE, None, 0, None, 0, None) == st
    # n_terms = 0 ignores the pointer
    plain = _prob(n=20, terms=FAKE + 4, n_terms=0)
    assert lib.qva_plan(ctypes.byref(plain), 2, 0, 0, None, 0) > 0


@pytest.mark.parametrize("n,p", [(13, 1), (20, 3), (28, 8)])
def test_zterm_plan(lib, n, p):
    """With terms the passes are those of QAOA; the phase passes read no q
    (first pass 16 B/amp, boundary 32 B/amp), and the gradient has one slot
    array per term and layer (workspace grows by p E tiles doubles) plus one
    array of 2^n doubles: each backward phase pass writes Im(conj(chi) phi)
    there instead of reading q, and a pass of kind 50 right after it turns
    those values into the per-term slots."""
    E = 37
    zt = _prob(n=n, terms=FAKE, n_terms=E)
    pl = _prob(n=n)
    N = 1 << n
    for flags in (0, 1):
        a = _plan(lib, n, p, flags=flags)
        cnt = lib.qva_plan(ctypes.byref(zt), p, 0, flags, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        assert lib.qva_plan(ctypes.byref(zt), p, 0, flags, arr, cnt) == cnt == len(a)
        for x, y in zip(arr, a):
            assert (x.kind, x.group_first, x.mix_layer, x.mix_layer2, x.phase_layer) == \
                   (y.kind, y.group_first, y.mix_layer, y.mix_layer2, y.phase_layer)
            assert x.bytes == y.bytes - (8 * N if y.kind in (1, 3) else 0)
    tiles = N >> 12
    w_plain = lib.qva_workspace_bytes(ctypes.byref(pl), p, 1)
    w_z = lib.qva_workspace_bytes(ctypes.byref(zt), p, 1)
    assert w_z - w_plain >= 8 * p * (E - 1) * tiles + 8 * N
    cnt = lib.qva_plan(ctypes.byref(zt), p, 1, 0, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(zt), p, 1, 0, arr, cnt) == cnt
    g = list(arr)
    gp = _grad_plan(lib, 0, n, p)
    # every backward phase pass (20, 21) is followed by a slot pass (50) over
    # the same tiles; without those the plan is the plain one
    zs = [i for i, x in enumerate(g) if x.kind == 50]
    assert len(zs) == p and all(g[i - 1].kind in (20, 21) for i in zs)
    for i in zs:
        assert (g[i].group_first, g[i].group_bits, g[i].col_bits, g[i].phase_layer) == \
               (g[i - 1].group_first, g[i - 1].group_bits, g[i - 1].col_bits, g[i - 1].phase_layer)
        assert g[i].bytes == 8 * N + 8 * E * tiles
    rest = [x for x in g if x.kind != 50]
    assert [x.kind for x in rest] == [x.kind for x in gp]
    for x, y in zip(rest, gp):
        if x.kind in (20, 21):  # Im(conj(chi) phi) written in place of the q read
            assert x.bytes == y.bytes
        elif x.kind == 25:      # the slot reduction covers p (G + E) slots
            assert x.bytes == y.bytes + 8 * p * (E - 1) * tiles
        else:
            assert x.bytes == y.bytes - (8 * N if x.kind in (1, 3) else 0)


# ------------------------------------------------------------------ QAOAz
def _xy_prob(n, pairs, q=FAKE, n_states=0):
    arr = None
    if pairs is not None:
        arr = (ctypes.c_int32 * (2 * max(1, len(pairs))))(*[x for pr in pairs for x in pr])
    pr = _lib.QvaProblem(2, n, q, None, 0, n_states, None, 0,
                         ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None,
                         len(pairs) if pairs is not None else 0)
    pr._keep = arr
    return pr


def _ring(m):
    from paper_2110_03963_amd import parity_ring_pairs
    return parity_ring_pairs(range(m))


def test_parity_ring_pairs(lib):
    """qva_parity_ring_pairs against the oracle's own construction of the
    parity mixer's factor order (eqs. parity_terms, qaoaz_mixers) for rings of
    2..15 qubits in natural and shuffled order; the sizing call, truncation
    and argument errors."""
    import numpy as np

    import oracle
    from paper_2110_03963_amd import parity_ring_pairs

    rng = np.random.default_rng(5)
    for m in range(2, 16):
        for ring in (list(range(m)), [int(x) for x in rng.permutation(24)[:m]]):
            ref = [tuple(int(v) for v in x) for x in oracle.parity_ring_pairs(ring)]
            assert parity_ring_pairs(ring) == ref, (m, ring)
            assert len(ref) == 2 * (m // 2) + (m % 2 == 1 and m >= 3)
    ring = (ctypes.c_int * 5)(4, 7, 1, 9, 2)
    assert lib.qva_parity_ring_pairs(ring, 5, None, 0) == 5
    out = (ctypes.c_int * 4)(-1, -1, -1, -1)
    assert lib.qva_parity_ring_pairs(ring, 5, out, 2) == 5  # first two pairs only
    assert list(out) == [4, 7, 1, 9]
    assert lib.qva_parity_ring_pairs(ring, 1, None, 0) == 0
    assert lib.qva_parity_ring_pairs(None, 0, None, 0) == 0
    S = _lib
    assert lib.qva_parity_ring_pairs(None, 3, None, 0) == S.QVA_ERR_ARG
    assert lib.qva_parity_ring_pairs(ring, -1, None, 0) == S.QVA_ERR_ARG
    assert lib.qva_parity_ring_pairs(ring, 5, None, 2) == S.QVA_ERR_ARG
    assert lib.qva_parity_ring_pairs(ring, 5, out, -1) == S.QVA_ERR_ARG


def test_xy_validation(lib):
    S = _lib
    assert S.QVA_MAX_XY_PAIRS == 256
    assert lib.qva_plan(ctypes.byref(_xy_prob(20, _ring(20))), 2, 0, 0, None, 0) > 0
    bad = [(_xy_prob(20, [(3, 3)]), S.QVA_ERR_ARG),
           (_xy_prob(20, [(0, 20)]), S.QVA_ERR_ARG),
           (_xy_prob(20, [(-1, 2)]), S.QVA_ERR_ARG),
           (_xy_prob(20, [(0, 1)] * 257), S.QVA_ERR_ARG),
           (_xy_prob(26, [(12, 24)]), S.QVA_ERR_UNSUPPORTED),   # no tile holds both
           (_xy_prob(17, _ring(17), n_states=100003), S.QVA_ERR_UNSUPPORTED)]
    nul = _lib.QvaProblem(2, 20, FAKE, None, 0, 0, None, 0, None, 3)
    bad.append((nul, S.QVA_ERR_ARG))
    zt = _lib.QvaProblem(2, 20, FAKE, None, 0, 0, FAKE, 3, None, 0)
    bad.append((zt, S.QVA_ERR_UNSUPPORTED))
    for pr, st in bad:
        assert lib.qva_plan(ctypes.byref(pr), 2, 0, 0, None, 0) == st
        assert lib.qva_workspace_bytes(ctypes.byref(pr), 2, 1) == 0
    # pairs that some tile holds: low qubit <= 10, or at most 8 apart
    assert lib.qva_plan(ctypes.byref(_xy_prob(30, [(10, 29), (20, 28), (0, 29)])), 1, 0, 0, None, 0) > 0
    # no pairs: the mixer is the identity, one phase pass per layer
    none = _xy_prob(20, [])
    assert lib.qva_plan(ctypes.byref(none), 3, 0, 0, None, 0) == 4


def _xy_plan(lib, pr, p, for_grad, flags=0):
    cnt = lib.qva_plan(ctypes.byref(pr), p, for_grad, flags, None, 0)
    assert cnt > 0
    arr = (_lib.QvaPassInfo * cnt)()
    assert lib.qva_plan(ctypes.byref(pr), p, for_grad, flags, arr, cnt) == cnt
    return list(arr)


@pytest.mark.parametrize("n,p", [(6, 2), (12, 1), (13, 3), (20, 2), (26, 3), (30, 2)])
def test_xy_plan(lib, n, p):
    """Each layer's passes apply all of its pair factors once, the phase only
    in the first; the gradient's walk inverts every forward pass; bytes and
    workspace follow the pass flags."""
    ring = _ring(n)
    pr = _xy_prob(n, ring)
    N = 1 << n
    for flags in (0, 1):
        plan = _xy_plan(lib, pr, p, 0, flags)
        assert plan[-1].kind == 8
        passes = plan[:-1]
        G = len(passes) // p
        assert len(passes) == G * p
        assert [x.kind for x in passes] == [42] * (G * p - 1) + [43]
        for k in range(p):
            layer = passes[k * G:(k + 1) * G]
            assert sum(x.mix_layer2 for x in layer) == len(ring)
            assert [x.phase_layer for x in layer] == [k] + [-1] * (G - 1)
            assert all(x.mix_layer == k for x in layer)
        for x in passes[:-1]:
            assert x.bytes == (32 + (8 if x.phase_layer >= 0 else 0)) * N
        last = passes[-1]
        assert last.bytes == (16 + 8 + (0 if flags else 16)) * N
    g = _xy_plan(lib, pr, p, 1)
    G = (len(g) - 2) // (2 * p)
    assert [x.kind for x in g] == [42] * (G * p - 1) + [44] + [45] * (G * p) + [8, 25]
    assert g[G * p - 1].bytes == (16 + 8 + 16 + 16) * N
    back = g[G * p:2 * G * p]
    assert [x.phase_layer for x in back] == [k if i == 0 else -1 for k in range(p - 1, -1, -1)
                                             for i in range(G - 1, -1, -1)]
    tiles = max(1, N >> 12)
    assert lib.qva_workspace_bytes(ctypes.byref(pr), p, 1) >= 16 * tiles + 8 * p * (G + 1) * tiles
    # depth 0: <psi0|Q|psi0> only
    assert [x.kind for x in _xy_plan(lib, pr, 0, 0)] == [7, 8]


# ------------------------------------------------------------ streaming probe
def test_stream_probe_rejects_bad_arguments():
    """The probe built with the library checks its arguments before touching
    the GPU: n outside 13..31 (13..30 with -2, two vectors) and tiles that do
    not fit the register exit with status 2 and a message."""
    import subprocess

    exe = os.path.join(ROOT, "paper_2110_03963_amd", "stream_probe")
    if not os.path.exists(exe):
        pytest.skip("probe not built")
    for args, msg in [(["40"], "n must be in 13..31"), (["-2", "31"], "n must be in 13..30"),
                      (["28", "4", "30"], "bad tile"), (["28", "2", "12"], "bad tile"),
                      (["-2", "20", "12", "11"], "bad tile")]:
        res = subprocess.run([exe] + args, capture_output=True, text=True, timeout=30)
        assert res.returncode == 2 and msg in res.stderr, (args, res.returncode, res.stderr)


def test_evolve_noalloc_validation(lib):
    """qva_evolve_noalloc reports argument errors and the static-scratch limit
    before it touches the device (fake pointers are never dereferenced)."""
    S = _lib
    ref = ctypes.byref
    big = _prob(n=33)  # 2^21 tiles of partial sums: 32 MiB > 16 MiB
    assert lib.qva_workspace_bytes(ref(big), 2, 0) > S.QVA_STATIC_SCRATCH_BYTES
    assert lib.qva_evolve_noalloc(ref(big), FAKE, FAKE, 2, FAKE, FAKE, None, 0, None) == S.QVA_ERR_SCRATCH
    ok = _prob(n=20)
    assert lib.qva_workspace_bytes(ref(ok), 2, 0) <= S.QVA_STATIC_SCRATCH_BYTES
    assert lib.qva_evolve_noalloc(ref(ok), FAKE, FAKE, 2, None, FAKE, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve_noalloc(ref(ok), FAKE, FAKE, 2, FAKE, None, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve_noalloc(ref(ok), None, FAKE, 2, FAKE, FAKE, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve_noalloc(ref(ok), FAKE, FAKE, 2, FAKE, FAKE, None, 4, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve_noalloc(None, FAKE, FAKE, 2, FAKE, FAKE, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_evolve_noalloc(ref(_prob(n=34)), FAKE, FAKE, 2, FAKE, FAKE, None, 0, None) == S.QVA_ERR_SIZE
    assert lib.qva_status_string(S.QVA_ERR_SCRATCH) == b"request needs more workspace than the static scratch holds"


def _factors(N):
    f, d = [], 2
    while d * d <= N:
        while N % d == 0:
            f.append(d)
            N //= d
        d += 1
    if N > 1:
        f.append(N)
    return f


@pytest.mark.parametrize("N", [6, 30, 1000, 3003, 6000, 3 * 2 ** 16, 243000, 184756, 460288, 2704156,
                               10400600, 11907000, 3 * 2 ** 29])
@pytest.mark.parametrize("p", [1, 4])
def test_plan_mixed_radix(lib, N, p):
    """N not a power of two with prime factors <= 31: the in-place mixed-radix
    passes.  The groups' sizes multiply to N within their caps (4096 for the
    contiguous group, 512 for strided ones), a tile holds at most 4096
    amplitudes, and the pass list is the power-of-two transform's: top group
    first, per layer the middle groups forward, the low group with the
    diagonal, the middle groups back, the boundary pass; the adjoint walks it
    back with one t slot and one gamma slot per layer."""
    n = (N - 1).bit_length()
    pr = _prob(mixer=1, n=n, kind=1, n_states=N)
    for grad in (0, 1):
        cnt = lib.qva_plan(ctypes.byref(pr), p, grad, 1, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        assert lib.qva_plan(ctypes.byref(pr), p, grad, 1, arr, cnt) == cnt
        kinds = [x.kind for x in arr]
        assert kinds[0] == 52 and not any(34 <= k <= 41 for k in kinds)
        groups = {}
        for x in arr:
            if x.group_first >= 0:
                groups[x.group_first] = (x.group_bits, x.col_bits)
        G = len(groups)
        assert sorted(groups) == list(range(G))
        prod = 1
        for g, (A, c) in groups.items():
            prod *= A
            assert A <= (4096 if g == 0 else 512) and A * c <= 4096 and c >= 1
        assert prod == N
        assert all(f <= 31 for f in _factors(N))
        if G == 1:
            assert kinds == [52, 67 if grad else 60]
            continue
        layer = [54] * (G - 2) + [56] + [55] * (G - 2)
        fwd = [53]
        for k in range(p):
            fwd += layer + ([57] if k + 1 < p else [58])
        if not grad:
            assert kinds == [52] + fwd + [8]
        else:
            back = []
            for k in range(p - 1, -1, -1):
                back += [62] * (G - 2) + [64] + [63] * (G - 2) + ([65] if k > 0 else [66])
            assert kinds == [52] + fwd[:-1] + [61] + back + [8, 25]
        assert lib.qva_workspace_bytes(ctypes.byref(pr), p, grad) > 0


def test_plan_large_prime_factor_stays_bluestein(lib):
    """A prime factor above 31 (4097 = 17 x 241, 1009 prime): Bluestein."""
    for N in (4097, 1009, 2 * 37 * 512):
        pr = _prob(mixer=1, n=(N - 1).bit_length(), kind=1, n_states=N)
        cnt = lib.qva_plan(ctypes.byref(pr), 2, 0, 1, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        lib.qva_plan(ctypes.byref(pr), 2, 0, 1, arr, cnt)
        kinds = [x.kind for x in arr]
        assert 52 not in kinds and 34 in kinds


def test_group_split_setting(lib):
    """qva_set_group_split validates the split and the planner follows it;
    count 0 restores the default (fewest groups of <= 9, near-equal)."""
    S = _lib
    IntArr = ctypes.c_int * 8
    out = IntArr()
    assert lib.qva_get_group_split(28, out, 8) == 2 and list(out)[:2] == [8, 8]
    assert lib.qva_get_group_split(12, out, 8) == 0
    assert lib.qva_set_group_split(28, IntArr(9, 7), 2) == S.QVA_OK
    try:
        assert lib.qva_get_group_split(28, out, 8) == 2 and list(out)[:2] == [9, 7]
        pr = _prob(n=28)
        cnt = lib.qva_plan(ctypes.byref(pr), 2, 0, 1, None, 0)
        arr = (_lib.QvaPassInfo * cnt)()
        lib.qva_plan(ctypes.byref(pr), 2, 0, 1, arr, cnt)
        groups = sorted({(x.group_first, x.group_bits, x.col_bits) for x in arr if x.group_first >= 0})
        assert groups == [(0, 12, 0), (12, 9, 3), (21, 7, 5)]
        assert lib.qva_set_group_split(28, IntArr(6, 5, 5), 3) == S.QVA_OK
        cnt = lib.qva_plan(ctypes.byref(pr), 2, 0, 1, None, 0)
        assert cnt == 2 * (4 - 1) + 1 + 1  # p (P - 1) + 1 passes and the reduction
    finally:
        assert lib.qva_set_group_split(28, None, 0) == S.QVA_OK
    assert lib.qva_get_group_split(28, out, 8) == 2 and list(out)[:2] == [8, 8]
    assert lib.qva_set_group_split(28, IntArr(10, 6), 2) == S.QVA_ERR_ARG   # a group above 9
    assert lib.qva_set_group_split(28, IntArr(8, 7), 2) == S.QVA_ERR_ARG    # sums to 15, not 16
    assert lib.qva_set_group_split(28, IntArr(0, 16), 2) == S.QVA_ERR_ARG
    assert lib.qva_set_group_split(12, IntArr(1), 1) == S.QVA_ERR_SIZE
    assert lib.qva_set_group_split(34, IntArr(9, 9, 4), 3) == S.QVA_ERR_SIZE
    assert lib.qva_set_group_split(28, None, 2) == S.QVA_ERR_ARG


def test_mix_circulant_validation(lib):
    """The lone circulant mixer takes every N >= 2 up to 2^33 for the
    complete graph, and for the ring and an eigenvalue array every power of
    two and every other N < 2^31 (mixed radix for prime factors <= 31, else
    Bluestein's transform); its workspace covers every eigenvalue kind.
    Arguments are checked before any launch."""
    S = _lib
    ring, array, complete = 1, 0, 2
    assert lib.qva_mix_circulant(None, None, ring, 1024, 0.1, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_mix_circulant(FAKE, None, array, 1024, 0.1, None, 0, None) == S.QVA_ERR_ARG
    assert lib.qva_mix_circulant(FAKE, None, ring, 1, 0.1, None, 0, None) == S.QVA_ERR_SIZE
    assert lib.qva_mix_circulant(FAKE, None, ring, -6, 0.1, None, 0, None) == S.QVA_ERR_SIZE
    big = (1 << 31) + 11  # a prime: neither mixed radix nor under Bluestein's 2^31
    assert lib.qva_mix_circulant(FAKE, None, ring, big, 0.1, FAKE, 1 << 40, None) == S.QVA_ERR_UNSUPPORTED
    assert lib.qva_mix_circulant(FAKE, None, complete, (1 << 33) + 1, 0.1, FAKE, 1 << 40, None) == S.QVA_ERR_SIZE
    assert lib.qva_mix_circulant_workspace_bytes((1 << 33) + 1) == 0
    # above 2^31 only the complete graph's per-block sums (4096 amplitudes a block), then S
    assert lib.qva_mix_circulant_workspace_bytes(big) == (16 * -(-big // 4096) + 255) // 256 * 256 + 256
    for N in (6, 1009, 6000, 2 * 37 * 512, 10400600, 3000017):
        ws = lib.qva_mix_circulant_workspace_bytes(N)
        assert ws > 0
        for kind, lam in ((ring, None), (array, FAKE), (complete, None)):
            assert lib.qva_mix_circulant(FAKE, lam, kind, N, 0.1, None, 0, None) == S.QVA_ERR_WORKSPACE
            assert lib.qva_mix_circulant(FAKE, lam, kind, N, 0.1, FAKE, ws - 1, None) == S.QVA_ERR_WORKSPACE
            assert lib.qva_mix_circulant(FAKE + 8, lam, kind, N, 0.1, FAKE, ws, None) == S.QVA_ERR_ALIGN
            assert lib.qva_mix_circulant(FAKE, lam, kind, N, 0.1, FAKE + 8, ws, None) == S.QVA_ERR_ALIGN
        assert lib.qva_mix_circulant(FAKE, FAKE + 4, array, N, 0.1, FAKE, ws, None) == S.QVA_ERR_ALIGN
    # Bluestein's buffers: the padded state and two filter spectra of M >= 2N - 1 amplitudes
    M = 1 << (2 * 3000017 - 2).bit_length()
    assert lib.qva_mix_circulant_workspace_bytes(3000017) >= 3 * M * 16
    assert lib.qva_mix_circulant_workspace_bytes(1 << 20) > 0
    assert lib.qva_mix_circulant_workspace_bytes(1 << 12) == 0


@pytest.mark.parametrize("N", [10400600, 11907000, 831600, 40116600, 155117520])
def test_mixed_radix_strided_rows_aligned(lib, N):
    """For these N (each with a fewest-group factorisation whose contiguous
    group holds 2^3) the planner takes such a factorisation and gives every
    strided group a multiple of 8 columns, so each row of a strided tile
    covers whole 128-byte lines (16 B per amplitude)."""
    n = (N - 1).bit_length()
    pr = _prob(mixer=1, n=n, kind=1, n_states=N)
    cnt = lib.qva_plan(ctypes.byref(pr), 1, 0, 1, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    lib.qva_plan(ctypes.byref(pr), 1, 0, 1, arr, cnt)
    groups = {x.group_first: (x.group_bits, x.col_bits) for x in arr if x.group_first >= 0}
    assert N % 8 == 0 and groups[0][0] % 8 == 0
    for g in range(1, len(groups)):
        A, cols = groups[g]
        assert cols % 8 == 0 and cols * A <= 4096 and cols >= 8, (g, A, cols)


def test_q_tiles_sizes_and_errors(lib):
    """qva_q_tiles_bytes / qva_q_tiles: one N-double block per qubit group for
    the hypercube mixer, 0 where no pass reads it; argument errors before any
    launch; a q_tiles key that does not match the split is rejected."""
    S = _lib
    key = ctypes.c_uint64(0)
    for n, groups in [(13, 2), (20, 2), (21, 2), (28, 3), (30, 3)]:
        pr = _prob(0, n)
        assert lib.qva_q_tiles_bytes(ctypes.byref(pr)) == groups * (1 << n) * 8
        # errors found before the device is touched
        assert lib.qva_q_tiles(ctypes.byref(pr), None, 1 << 40, ctypes.byref(key), None) == S.QVA_ERR_ARG
        assert lib.qva_q_tiles(ctypes.byref(pr), FAKE, 1 << 40, None, None) == S.QVA_ERR_ARG
        assert lib.qva_q_tiles(ctypes.byref(pr), FAKE + 4, 1 << 40, ctypes.byref(key), None) == S.QVA_ERR_ALIGN
        assert lib.qva_q_tiles(ctypes.byref(pr), FAKE, groups * (8 << n) - 8, ctypes.byref(key),
                               None) == S.QVA_ERR_WORKSPACE
    # no pass reads the copy: small registers, circulant mixers, Z-string terms
    for pr in [_prob(0, 12), _prob(1, 20, kind=1), _prob(0, 20, terms=FAKE, n_terms=3)]:
        assert lib.qva_q_tiles_bytes(ctypes.byref(pr)) == 0
        assert lib.qva_q_tiles(ctypes.byref(pr), FAKE, 1 << 40, ctypes.byref(key), None) == S.QVA_ERR_UNSUPPORTED
    assert lib.qva_q_tiles(None, FAKE, 1 << 40, ctypes.byref(key), None) == S.QVA_ERR_ARG
    # a descriptor carrying a copy with a wrong key or a misaligned copy
    stale = _prob(0, 20)
    stale.q_tiles = FAKE
    stale.q_tiles_key = 12345
    assert lib.qva_plan(ctypes.byref(stale), 2, 0, 0, None, 0) == S.QVA_ERR_ARG
    assert lib.qva_workspace_bytes(ctypes.byref(stale), 2, 1) == 0
    # sizing and rewriting look past the descriptor's own (stale) copy
    assert lib.qva_q_tiles_bytes(ctypes.byref(stale)) == 2 * (1 << 20) * 8
    assert lib.qva_q_tiles(ctypes.byref(stale), FAKE, 8, ctypes.byref(key), None) == S.QVA_ERR_WORKSPACE
    stale.q_tiles = FAKE + 4
    assert lib.qva_plan(ctypes.byref(stale), 2, 0, 0, None, 0) == S.QVA_ERR_ALIGN
    # mixers that never read it ignore it, key and all
    circ = _prob(1, 20, kind=1)
    circ.q_tiles = FAKE + 4
    circ.q_tiles_key = 12345
    assert lib.qva_plan(ctypes.byref(circ), 2, 0, 0, None, 0) > 0
