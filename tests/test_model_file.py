"""Persisted HARP models (a model is built once per element and frequency and
reused for any layout, Section III-C): save / load round trip of the blob,
and rejection of a wrong magic, version, size, a corrupted sample copy and a
different element.  CPU only (the blob is host memory here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import em, fit as ofit  # noqa: E402
from workloads import element  # noqa: E402


@pytest.fixture(scope="module")
def model():
    from paper_1702_03781_amd import api
    el = element(3, 9, seed=77)
    m = ofit.fit(120e6, el.samples, 6, 6, 1.5, wire_radius=el.wire_radius)
    return el, api.pack_model(m.C, m.Z_self, m.w, m.samples, m.freq, m.k, em.omega_mu(m.freq), m.r_min,
                              m.wire_radius, device="cpu")


def test_round_trip(tmp_path, model):
    from paper_1702_03781_amd import api
    el, m = model
    p = str(tmp_path / "m.harp")
    api.save_model(m, p)
    back = api.load_model(p, device="cpu", samples=el.samples, wire_radius=el.wire_radius)
    assert torch.equal(back.blob, m.blob)
    assert (back.n_mbf, back.n_samp, back.P, back.Q, back.freq, back.r_min) == \
        (m.n_mbf, m.n_samp, m.P, m.Q, m.freq, m.r_min)
    assert back.reciprocal and m.reciprocal
    arrays = api.model_arrays(back)
    assert arrays["C"].shape == (3, 3, 13, 7)
    assert api.model_layout_bytes(3, 9, 6, 6) == api.model_bytes(3, 9, 6, 6) == m.nbytes


def _corrupt(src, dst, offset, data):
    raw = bytearray(open(src, "rb").read())
    raw[offset:offset + len(data)] = data
    open(dst, "wb").write(bytes(raw))


def test_rejections(tmp_path, model):
    from paper_1702_03781_amd import api
    el, m = model
    p = str(tmp_path / "m.harp")
    api.save_model(m, p)
    hdr = 56                                    # file header bytes
    cases = {
        "magic": (0, b"NOTHARP!"),
        "version": (8, (99).to_bytes(4, "little")),
        "blob magic": (hdr, b"\0\0\0\0"),
        "sample copy": (hdr + int(api.read_model_header(m)["off_samples"]) + 3, b"\x7f"),
    }
    for name, (off, data) in cases.items():
        q = str(tmp_path / f"bad_{name.replace(' ', '_')}.harp")
        _corrupt(p, q, off, data)
        with pytest.raises(ValueError):
            api.load_model(q, device="cpu")
    # truncated blob
    q = str(tmp_path / "short.harp")
    open(q, "wb").write(open(p, "rb").read()[:-16])
    with pytest.raises(ValueError):
        api.load_model(q, device="cpu")
    # a different element
    other = element(3, 9, seed=78)
    with pytest.raises(ValueError):
        api.load_model(p, device="cpu", samples=other.samples, wire_radius=other.wire_radius)
    with pytest.raises(ValueError):
        api.load_model(p, device="cpu", samples=el.samples, wire_radius=el.wire_radius * 2)


def test_pack_model_flags_nonreciprocal_tables(model):
    from paper_1702_03781_amd import api
    el, m = model
    arrays = api.model_arrays(m)
    C = arrays["C"].copy()
    C[0, 1, 2, 3] += 1e-3 * np.abs(C).max()
    h = arrays["header"]
    bad = api.pack_model(C, arrays["Z_self"], arrays["w"], el.samples, h["freq_hz"], h["k"], h["omega_mu"],
                         h["r_min"], h["wire_radius"], device="cpu")
    assert not bad.reciprocal
