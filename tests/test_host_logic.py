"""Host checks of index identities the kernels rely on (no GPU needed).

* Three-column tiles rotate element bit 3 across lanes: the partner of lane
  i is read with DPP row_mirror (lane ^ 15 within each row of 16) followed by
  row_half_mirror (lane ^ 7 within each half row); the composition must be
  lane ^ 8 for all 64 lanes, and element bit 3 must be lane bit 3 in the
  layouts where the rotation runs (A: e = t | r << 8; B: e = (t & 15) |
  r << 4 | (t >> 4) << 8).
* The ring diagonal of the low-group transform pass pairs registers r and
  r + 1 (r even): their digits k = rev4(r) and rev4(r + 1) differ by 8, so
  the eigenvalues 2 Re(u conj(W_16^k)) are exact negatives.
"""


def _row_mirror(i):
    return (i & ~15) | (15 - (i & 15))


def _row_half_mirror(i):
    return (i & ~7) | (7 - (i & 7))


def test_dpp_mirror_composition_is_xor8():
    for lane in range(64):
        # value after the first step at lane j is the source at mirror(j); after
        # the second, lane i holds the first step's value at half_mirror(i)
        src = _row_mirror(_row_half_mirror(lane))
        assert src == lane ^ 8, lane


def test_element_bit3_is_lane_bit3_in_layouts_a_and_b():
    for t in range(256):
        for r in range(16):
            ea = t | (r << 8)
            eb = (t & 15) | (r << 4) | ((t >> 4) << 8)
            assert (ea >> 3) & 1 == (t >> 3) & 1
            assert (eb >> 3) & 1 == (t >> 3) & 1
            # the lane partner (t ^ 8) holds the element with bit 3 flipped
            assert ((t ^ 8) | (r << 8)) == ea ^ 8
            assert (((t ^ 8) & 15) | (r << 4) | (((t ^ 8) >> 4) << 8)) == eb ^ 8


def _rev4(x):
    return int(f"{x:04b}"[::-1], 2)


def test_ring_digit_pairs_differ_by_eight():
    import math

    for r in range(0, 16, 2):
        k0, k1 = _rev4(r), _rev4(r + 1)
        assert k1 == k0 + 8 and k0 < 8
        # W_16^(k+8) = -W_16^k, so the eigenvalues are negatives for any u
        for ang in (0.1, 1.3, 2.9):
            u = complex(math.cos(ang), math.sin(ang))
            w0 = complex(math.cos(2 * math.pi * k0 / 16), -math.sin(2 * math.pi * k0 / 16))
            w1 = complex(math.cos(2 * math.pi * k1 / 16), -math.sin(2 * math.pi * k1 / 16))
            l0 = 2 * (u * w0.conjugate()).real
            l1 = 2 * (u * w1.conjugate()).real
            assert abs(l0 + l1) < 1e-14


def test_grad_rejects_short_state_before_any_launch(monkeypatch):
    """grad() checks that psi and chi hold N amplitudes before it calls the
    library (qva_grad writes N amplitudes into both)."""
    import torch

    import paper_2110_03963_amd.qva as qmod

    def no_library():
        raise AssertionError("the library was called")

    monkeypatch.setattr(qmod, "_need", lambda t, dtype, name: None)
    monkeypatch.setattr(qmod._lib, "load", no_library)
    prob = object.__new__(qmod.Problem)
    prob._N = 16
    prob.q = torch.zeros(16, dtype=torch.float64)
    prob.n_terms = 0
    prob.psi0 = None
    good = torch.zeros(16, dtype=torch.complex128)
    short = torch.zeros(15, dtype=torch.complex128)
    for psi, chi in ((short, good), (good, short), (short, short)):
        try:
            qmod.grad(prob, [0.1], [0.2], psi=psi, chi=chi)
        except ValueError as e:
            assert "N amplitudes" in str(e)
        else:
            raise AssertionError("no ValueError for a short psi/chi")
