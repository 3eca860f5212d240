"""MLP weight fragments as the library stages them for the matrix cores
(host only; no GPU): the FP32 engine's three BF16 pieces of each weight add
up to it exactly, and the BF16 engine's single piece is the weight rounded
to nearest even.  Checked per layer as multisets, which leaves the lane
layout to the GPU parity tests."""
import numpy as np
import pytest

from paper_2309_04581_amd import scenegen as sg


def mr():
    from paper_2309_04581_amd import meshrf as M
    M.lib()
    return M


def bf16_halves(words):
    """uint32 words -> the two bf16 values each holds, as float64 (low half first)."""
    w = np.asarray(words, dtype=np.uint32)
    lo = (w & 0xFFFF).astype(np.uint32) << 16
    hi = w & 0xFFFF0000
    vals = np.stack([lo, hi], axis=-1).reshape(-1)
    return vals.view(np.float32).astype(np.float64)


def rne_bf16(x):
    """Round float32 values to bf16 (nearest even) by their bit patterns."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def layers(f):
    """(name, weights) of the layers staged as BF16 fragments, in staging order."""
    m = np.asarray(f.mlp, dtype=np.float32)
    o = 0
    W1 = m[o:o + 64 * f.d_in].reshape(64, f.d_in); o += 64 * f.d_in
    W2 = m[o:o + 16 * 64]; o += 16 * 64
    Wc1 = m[o:o + 64 * f.c_in].reshape(64, f.c_in); o += 64 * f.c_in
    nfeat = f.n_levels * f.feats       # inputs past the features are zero padding, not staged
    out = [("density 1", W1[:, :nfeat].reshape(-1)), ("density 2", W2),
           ("colour 1 (raw inputs)", Wc1[:, :16].reshape(-1))]
    if f.c_layers == 2:
        out.append(("colour 2", m[o:o + 64 * 64]))
    return out


@pytest.mark.parametrize("make", [sg.mid_field, sg.tiny_field])
def test_fp32_fragments_are_exact_three_piece_splits(make):
    M = mr()
    f = make()
    fr = M.mr_mlp_fragments(f, bf16=False)
    off = 0
    for name, w in layers(f):
        n_words = w.size // 2          # two bf16 values per word, one piece
        pieces = [bf16_halves(fr[off + q * n_words: off + (q + 1) * n_words]) for q in range(3)]
        off += 3 * n_words
        p0, p1, p2 = pieces
        total = p0 + p1 + p2           # exact in float64: 3 x 8 significant bits
        np.testing.assert_array_equal(np.sort(total), np.sort(w.astype(np.float64)), err_msg=name)
        # the pieces are the successive nearest-even roundings of the residuals
        order = np.argsort(total, kind="stable")
        ws = np.sort(w.astype(np.float64), kind="stable")
        assert np.all(p0[order] == rne_bf16(ws)), name
        r1 = (ws - rne_bf16(ws)).astype(np.float32)
        assert np.all(p1[order] == rne_bf16(r1)), name
        assert np.all(np.abs(p2) <= np.abs(p1) * 2.0 ** -7 + 0.0), name
    # then the FP32 output layer and SH columns
    assert fr.size == off + 192 + 64 * f.sh


@pytest.mark.parametrize("make", [sg.mid_field, sg.tiny_field])
def test_bf16_fragments_are_rounded_weights(make):
    M = mr()
    f = make()
    fr = M.mr_mlp_fragments(f, bf16=True)
    off = 0
    for name, w in layers(f):
        n_words = w.size // 2
        got = bf16_halves(fr[off:off + n_words])
        off += n_words
        np.testing.assert_array_equal(np.sort(got), np.sort(rne_bf16(w)), err_msg=name)
    assert fr.size == off + 192 + 64 * f.sh


def test_fragment_export_validates():
    M = mr()
    f = sg.mid_field()
    d, res = M.field_desc(f)
    mlp = np.ascontiguousarray(f.mlp, dtype=np.float32)
    import ctypes as C
    words = C.c_int64()
    small = np.zeros(8, dtype=np.uint32)
    st = M.lib().mr_mlp_fragments(C.byref(d), M._ptr(mlp), C.c_int32(0), M._ptr(small), C.c_int64(8),
                                  C.byref(words))
    assert st != M.MR_OK and words.value > 8 and np.all(small == 0)
    # a proposal field has no fragments
    p = sg.make_proposal()
    dp, rp = M.field_desc(p)
    st = M.lib().mr_mlp_fragments(C.byref(dp), M._ptr(np.ascontiguousarray(p.mlp, dtype=np.float32)), C.c_int32(0),
                                  None, C.c_int64(0), C.byref(words))
    assert st != M.MR_OK
