"""Authenticated FITS container, plain Python over the CPU oracle's GCM --
TEST INFRASTRUCTURE ONLY (imported by tests/ alone; shares no code with the
product library).

What it writes, following the paper's "Authenticated FITS File Format",
"Context Binding via Associated Data (AAD)" and "Policy Enforcement and
Granular Access" sections, with the readings listed in the design notes:

* HDU 0 (NAXIS = 0): SIMPLE, BITPIX = 8, NAXIS = 0, EXTEND, LONGSTRN, NONCE_H
  and NONCE_D (upper-case hex), ORIG_BPX / ORIG_NAX / ORIG_NA1 / ORIG_NA2 (the
  original BITPIX, NAXIS, NAXIS1, NAXIS2), HIERARCH AUTHTAG_H / AUTHTAG_D
  (hex), ENCHDR: base64 of the GCM encryption of the original header blocks
  under the header key with AAD = NONCE_H, split in 64-character pieces over
  CONTINUE cards, then END.
* HDU 1: a BINTABLE with one row and one column (TTYPE1 = 'BLOB', TFORM1 =
  '<N>B') holding the GCM encryption of the N pixel bytes under the data key
  with AAD_D = NONCE_D || ascii(BITPIX) || ascii(NAXIS) || ascii(NAXIS1) ||
  ascii(NAXIS2).
* Decryption: header key wrong or missing -> a minimal header from ORIG_*
  (warning 1); data key wrong or missing, or the AAD's inputs changed ->
  zero pixels (warning 2); both -> 3.
"""
from __future__ import annotations

import numpy as np

from . import gcm_decrypt_verify, gcm_encrypt

CARD = 80
BLOCK = 2880


def serialize(v: int) -> bytes:
    """Strict ASCII decimal (the paper's example: -32 -> b'-32')."""
    return str(int(v)).encode("ascii")


def data_aad(nonce_d: bytes, bitpix: int, naxis: int, naxis1: int, naxis2: int) -> bytes:
    return bytes(nonce_d) + serialize(bitpix) + serialize(naxis) + serialize(naxis1) + serialize(naxis2)


def _pad(b: bytes, fill: bytes) -> bytes:
    return b + fill * ((-len(b)) % BLOCK)


def _card(text: str) -> str:
    assert len(text) <= CARD, text
    return text.ljust(CARD)


def _kw(name: str) -> str:
    return name.ljust(8) + "= "


def _int(name: str, v: int) -> str:
    return _card(_kw(name) + str(v).rjust(20))


def _log(name: str, v: bool) -> str:
    return _card(_kw(name) + ("T" if v else "F").rjust(20))


def _str(name: str, v: str) -> str:
    return _card(_kw(name) + "'" + v.ljust(8) + "'")


def _header(cards) -> bytes:
    return _pad("".join(cards + [_card("END")]).encode("ascii"), b" ")


def _b64(data: bytes) -> str:
    alphabet = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
    out = []
    for i in range(0, len(data), 3):
        chunk = data[i:i + 3]
        w = int.from_bytes(chunk + bytes(3 - len(chunk)), "big")
        sym = [alphabet[(w >> s) & 63] for s in (18, 12, 6, 0)]
        if len(chunk) < 3:
            sym[3] = "="
        if len(chunk) < 2:
            sym[2] = "="
        out.append("".join(sym))
    return "".join(out)


def parse_header(buf: bytes, off: int = 0):
    """(list of 80-char cards up to and including END, header size in bytes)."""
    cards = []
    p = off
    while p + CARD <= len(buf):
        c = buf[p:p + CARD].decode("ascii")
        cards.append(c)
        p += CARD
        if c.startswith("END     "):
            size = p - off
            return cards, size + (-size) % BLOCK
    raise ValueError("no END card")


def _value(cards, name):
    key = _kw(name)[:9]
    for c in cards:
        if c.startswith(key):
            return c[10:].split("/")[0].strip()
    raise KeyError(name)


def _string(cards, name):
    v = _value(cards, name)
    assert v.startswith("'")
    return v[1:v.index("'", 1)].strip()


def _hierarch(cards, name):
    key = "HIERARCH " + name + " = '"
    for c in cards:
        if c.startswith(key):
            return c[len(key):c.index("'", len(key))]
    raise KeyError(name)


def _long_string(cards, name):
    key = _kw(name)
    for i, c in enumerate(cards):
        if c.startswith(key):
            parts = []
            s = c[10:]
            j = i
            while True:
                body = s[1:s.index("'", 1)]
                if body.endswith("&"):
                    parts.append(body[:-1])
                    j += 1
                    s = cards[j][10:]
                    assert cards[j].startswith("CONTINUE  ")
                else:
                    parts.append(body)
                    return "".join(parts)
    raise KeyError(name)


def image_structure(fits: bytes):
    cards, hsize = parse_header(fits)
    bitpix, naxis = int(_value(cards, "BITPIX")), int(_value(cards, "NAXIS"))
    n1, n2 = int(_value(cards, "NAXIS1")), int(_value(cards, "NAXIS2"))
    return cards, hsize, bitpix, naxis, n1, n2


def encrypt(fits: bytes, key_h: bytes, key_d: bytes, nonce_h: bytes, nonce_d: bytes) -> bytes:
    cards, hsize, bitpix, naxis, n1, n2 = image_structure(fits)
    nd = abs(bitpix) // 8 * n1 * n2
    header = fits[:hsize]
    pixels = np.frombuffer(fits[hsize:hsize + nd], dtype=np.uint8)
    ct_h, tag_h = gcm_encrypt(key_h, nonce_h, nonce_h, np.frombuffer(header, np.uint8))
    ct_d, tag_d = gcm_encrypt(key_d, nonce_d, data_aad(nonce_d, bitpix, naxis, n1, n2), pixels)
    hdu0 = [_log("SIMPLE", True), _int("BITPIX", 8), _int("NAXIS", 0), _log("EXTEND", True),
            _str("LONGSTRN", "OGIP 1.0"), _str("NONCE_H", nonce_h.hex().upper()),
            _str("NONCE_D", nonce_d.hex().upper()), _int("ORIG_BPX", bitpix), _int("ORIG_NAX", naxis),
            _int("ORIG_NA1", n1), _int("ORIG_NA2", n2),
            _card("HIERARCH AUTHTAG_H = '" + tag_h.hex().upper() + "'"),
            _card("HIERARCH AUTHTAG_D = '" + tag_d.hex().upper() + "'")]
    enc = _b64(ct_h.tobytes())
    pieces = [enc[i:i + 64] for i in range(0, len(enc), 64)] or [""]
    for k, piece in enumerate(pieces):
        text = piece + ("&" if k + 1 < len(pieces) else "")
        hdu0.append(_card(("ENCHDR  = '" if k == 0 else "CONTINUE  '") + text + "'"))
    hdu1 = [_str("XTENSION", "BINTABLE"), _int("BITPIX", 8), _int("NAXIS", 2), _int("NAXIS1", nd),
            _int("NAXIS2", 1), _int("PCOUNT", 0), _int("GCOUNT", 1), _int("TFIELDS", 1), _str("TTYPE1", "BLOB"),
            _str("TFORM1", f"{nd}B")]
    return _header(hdu0) + _header(hdu1) + _pad(ct_d.tobytes(), b"\0")


def decrypt(container: bytes, key_h: bytes | None, key_d: bytes | None):
    """(FITS bytes, warning code).  The blob length comes from the BINTABLE;
    the AAD from the plaintext ORIG_* cards; the output pixels follow the
    structure of the output header (the authenticated original, else the
    minimal one built from ORIG_*)."""
    import base64  # only to decode what the oracle's own encoder wrote

    cards0, size0 = parse_header(container)
    cards1, size1 = parse_header(container, size0)
    bitpix, naxis = int(_value(cards0, "ORIG_BPX")), int(_value(cards0, "ORIG_NAX"))
    n1, n2 = int(_value(cards0, "ORIG_NA1")), int(_value(cards0, "ORIG_NA2"))
    nonce_h, nonce_d = bytes.fromhex(_string(cards0, "NONCE_H")), bytes.fromhex(_string(cards0, "NONCE_D"))
    tag_h, tag_d = bytes.fromhex(_hierarch(cards0, "AUTHTAG_H")), bytes.fromhex(_hierarch(cards0, "AUTHTAG_D"))
    ct_h = base64.b64decode(_long_string(cards0, "ENCHDR"))
    nblob = int(_value(cards1, "NAXIS1"))
    assert _string(cards1, "TFORM1") == f"{nblob}B"
    ct_d = np.frombuffer(container[size0 + size1:size0 + size1 + nblob], dtype=np.uint8)
    warn = 0
    header = None
    if key_h is not None and len(key_h) in (16, 24, 32):
        pt, ok = gcm_decrypt_verify(key_h, nonce_h, nonce_h, np.frombuffer(ct_h, np.uint8), tag_h)
        header = pt.tobytes() if ok else None
    if header is not None:
        _, _, obp, onax, on1, on2 = image_structure(header)
    else:
        header = _header([_log("SIMPLE", True), _int("BITPIX", bitpix), _int("NAXIS", naxis), _int("NAXIS1", n1),
                          _int("NAXIS2", n2)])
        obp, on1, on2 = bitpix, n1, n2
        warn |= 1
    nout = abs(obp) // 8 * on1 * on2
    pixels = None
    if key_d is not None and len(key_d) in (16, 24, 32):
        pt, ok = gcm_decrypt_verify(key_d, nonce_d, data_aad(nonce_d, bitpix, naxis, n1, n2), ct_d, tag_d)
        pixels = pt.tobytes() if ok and nblob == nout else None
    if pixels is None:
        pixels = bytes(nout)
        warn |= 2
    return header + _pad(pixels, b"\0"), warn
