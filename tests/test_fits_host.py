"""FITS export checked against the standard's layout (FITS 4.0: 2880-byte blocks,
80-character cards, mandatory keywords in order, END, big-endian IEEE data,
axis 1 fastest), read back by a reader written here from those rules."""
import numpy as np
import pytest

from paper_1904_11422_amd import fits


def _read(path):
    raw = open(path, "rb").read()
    assert len(raw) % 2880 == 0
    cards, pos = [], 0
    while True:
        card = raw[pos:pos + 80].decode("ascii")
        pos += 80
        cards.append(card)
        if card.startswith("END"):
            break
    hdr_end = (pos + 2879) // 2880 * 2880
    assert raw[pos:hdr_end] == b" " * (hdr_end - pos)
    kv = {}
    for c in cards[:-1]:
        key = c[:8].strip()
        assert c[8:10] == "= "
        val = c[10:].split(" / ")[0].strip()
        if val.startswith("'"):
            val = val.strip("'").rstrip()
        elif val in ("T", "F"):
            val = val == "T"
        elif "." in val or "E" in val:
            val = float(val)
        else:
            val = int(val)
        kv[key] = val
    return cards, kv, raw[hdr_end:]


@pytest.mark.parametrize("bitpix", [-32, -64])
def test_fits_cube_round_trip(tmp_path, bitpix):
    rng = np.random.default_rng(1)
    cube = rng.normal(size=(3, 4, 8, 8))
    freq = 38e6 + 25e3 * np.arange(3)
    p = tmp_path / "cube.fits"
    fits.write(str(p), cube, grid_n=8, cell_wavelengths=0.5, freq_hz=freq, bitpix=bitpix,
               n_time=1000, sample_s=40e-6)
    cards, kv, body = _read(str(p))
    assert [c[:8].strip() for c in cards[:7]] == ["SIMPLE", "BITPIX", "NAXIS", "NAXIS1",
                                                   "NAXIS2", "NAXIS3", "NAXIS4"]
    assert kv["SIMPLE"] is True and kv["BITPIX"] == bitpix and kv["NAXIS"] == 4
    assert (kv["NAXIS1"], kv["NAXIS2"], kv["NAXIS3"], kv["NAXIS4"]) == (8, 8, 4, 3)
    assert kv["CTYPE3"] == "STOKES" and kv["CRVAL3"] == 1.0
    assert kv["CTYPE4"] == "FREQ" and kv["CRVAL4"] == 38e6 and kv["CDELT4"] == 25e3
    assert kv["CRPIX1"] == 5.0 and kv["CDELT1"] == 0.25
    assert kv["NSAMPLES"] == 1000
    n = cube.size * (4 if bitpix == -32 else 8)
    assert body[n:] == b"\0" * (len(body) - n)
    got = np.frombuffer(body[:n], dtype=">f4" if bitpix == -32 else ">f8").reshape(3, 4, 8, 8)
    want = cube.astype(np.float32) if bitpix == -32 else cube
    assert np.array_equal(got, want)
    # axis 1 varies fastest: the second value in the file is pixel (m=0, l=1)
    assert got.reshape(-1)[1] == want[0, 0, 0, 1]


def test_fits_single_plane_and_refusals(tmp_path):
    p = tmp_path / "xx.fits"
    fits.write(str(p), np.ones((1, 4, 4)), grid_n=4)
    _, kv, _ = _read(str(p))
    assert kv["NAXIS"] == 3 and kv["CRVAL3"] == -5.0
    with pytest.raises(ValueError):
        fits.write(str(p), np.ones((2, 4, 4, 4)), grid_n=4, freq_hz=[1.0, 2.0, 4.0])
    with pytest.raises(ValueError):
        fits.write(str(p), np.ones((3, 4, 4, 4)), grid_n=4, freq_hz=[1.0, 2.0, 4.0])
    with pytest.raises(ValueError):
        fits.write(str(p), np.ones((4, 4)), grid_n=4, bitpix=16)
