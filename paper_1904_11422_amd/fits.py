"""FITS export of post-processed images (the paper's images are written to disk
and converted to FITS after the real-time path, Sec. 3.2).

A single primary HDU per file, following the FITS standard (version 4.0):
80-character ASCII header cards in 2880-byte blocks ending with END, then the
data array big-endian in 2880-byte blocks (IEEE float, BITPIX -32 or -64),
axis 1 varying fastest.  Axes of an image cube [C][S][N][N] (as
Imager.postprocess returns it): 1 = l and 2 = m (direction cosines, pixel
N/2 + 1 at zero, spacing 1 / (N * cell_wavelengths)), 3 = STOKES (1..4 =
I, Q, U, V; a single XX plane is labelled -5, the FITS code of XX), 4 = FREQ
(Hz, uniform channel spacing).  No celestial projection is written: the
imager knows the array, not the observing time and site.
"""
from __future__ import annotations

import numpy as np

_BLOCK = 2880


def _card(key: str, value=None, comment: str = "") -> bytes:
    """One 80-character header card (fixed format for the values used here)."""
    if value is None:
        text = f"{key:<8}"
    else:
        if isinstance(value, bool):
            v = f"{'T' if value else 'F':>20}"
        elif isinstance(value, (int, np.integer)):
            v = f"{int(value):>20d}"
        elif isinstance(value, (float, np.floating)):
            t = f"{float(value):.13G}"
            if "." not in t and "E" not in t:
                t += ".0"                       # keep it a real value
            v = f"{t:>20}"
        else:
            s = str(value).replace("'", "''")
            v = f"'{s:<8}'"
        text = f"{key:<8}= {v}"
        if comment:
            text += f" / {comment}"
    if len(text) > 80:
        raise ValueError(f"header card too long: {text!r}")
    return f"{text:<80}".encode("ascii")


def header_cards(shape, bitpix: int, grid_n: int, cell_wavelengths: float, freq_hz,
                 n_time: int = 0, sample_s: float = 0.0, extra=None) -> list:
    """The cards of a primary header for an image cube of the given numpy shape
    ([C][S][N][N]; C and S may be absent)."""
    naxis = len(shape)
    cards = [_card("SIMPLE", True, "conforms to FITS standard"),
             _card("BITPIX", bitpix, "IEEE floating point"),
             _card("NAXIS", naxis)]
    for i in range(naxis):
        cards.append(_card(f"NAXIS{i + 1}", int(shape[naxis - 1 - i])))
    d = 1.0 / (grid_n * cell_wavelengths)
    cards += [_card("CTYPE1", "L", "direction cosine, east"),
              _card("CRPIX1", grid_n / 2 + 1.0), _card("CRVAL1", 0.0), _card("CDELT1", d),
              _card("CTYPE2", "M", "direction cosine, north"),
              _card("CRPIX2", grid_n / 2 + 1.0), _card("CRVAL2", 0.0), _card("CDELT2", d)]
    if naxis >= 3:
        n_s = int(shape[naxis - 3])
        cards += [_card("CTYPE3", "STOKES"), _card("CRPIX3", 1.0),
                  _card("CRVAL3", 1.0 if n_s == 4 else -5.0), _card("CDELT3", 1.0)]
    if naxis >= 4:
        f = np.asarray(freq_hz, dtype=np.float64)
        df = float(f[1] - f[0]) if f.size > 1 else 1.0
        if f.size > 1 and np.max(np.abs(np.diff(f) - df)) > 1e-6 * abs(df):
            raise ValueError("FREQ axis needs uniformly spaced channels")
        cards += [_card("CTYPE4", "FREQ"), _card("CRPIX4", 1.0), _card("CRVAL4", float(f[0])),
                  _card("CDELT4", df), _card("CUNIT4", "Hz")]
    if n_time:
        cards.append(_card("NSAMPLES", int(n_time), "samples accumulated"))
    if sample_s:
        cards.append(_card("TSAMPLE", float(sample_s), "seconds per sample"))
    for k, v in (extra or {}).items():
        cards.append(_card(k, v))
    cards.append(_card("END"))
    return cards


def write(path: str, data, grid_n: int, cell_wavelengths: float = 0.5, freq_hz=None,
          bitpix: int = -32, n_time: int = 0, sample_s: float = 0.0, extra=None) -> None:
    """Write an image cube (numpy array or CPU/GPU tensor [C][S][N][N],
    [S][N][N] or [N][N]) as a FITS primary HDU."""
    if hasattr(data, "detach"):
        data = data.detach().cpu().numpy()
    arr = np.asarray(data)
    if bitpix not in (-32, -64):
        raise ValueError("bitpix must be -32 or -64")
    if arr.ndim == 4 and (freq_hz is None or len(freq_hz) != arr.shape[0]):
        raise ValueError("a 4-D cube needs one frequency per channel")
    cards = header_cards(arr.shape, bitpix, grid_n, cell_wavelengths, freq_hz, n_time, sample_s,
                         extra)
    head = b"".join(cards)
    head += b" " * (-len(head) % _BLOCK)
    body = np.ascontiguousarray(arr, dtype=">f4" if bitpix == -32 else ">f8").tobytes()
    body += b"\0" * (-len(body) % _BLOCK)
    with open(path, "wb") as fh:
        fh.write(head)
        fh.write(body)
