"""Seeded synthetic inputs with the shapes of the paper's workloads.

No cryptographic arithmetic lives here: only random bytes, keys, IVs and
FITS-shaped images, all drawn from numpy PCG64 streams spawned from one
master seed, so the GPU tests, the benchmark and the CPU oracle see the same
bytes.

FITS-shaped data follows the paper's synthetic dataset description (its
"Datasets" appendix table: float32 images of Gaussian sky noise) and the
workload sizes used here: BITPIX = -32 pixels stored big-endian, the data
unit zero-padded to a multiple of 2880 bytes, point sources with the FWHM
the paper's photometric check reports (6.84 px), and a 2880-byte ASCII
header of 80-character cards used as the associated data.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

FITS_BLOCK = 2880
CARD = 80


def rng_for(seed: int, *path: int) -> np.random.Generator:
    """Independent stream for (seed, path...)."""
    ss = np.random.SeedSequence([seed, *path])
    return np.random.Generator(np.random.PCG64(ss))


def random_bytes(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 256, size=n, dtype=np.uint8)


def fits_header(rng: np.random.Generator, cards: int = 36) -> bytes:
    """`cards`-1 random keyword cards plus an END card: 80 ASCII chars each."""
    alnum = np.frombuffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZ0123456789_", dtype=np.uint8)
    out = bytearray()
    for _ in range(cards - 1):
        kw = bytes(alnum[rng.integers(0, len(alnum), 8)])
        val = bytes(rng.integers(0x20, 0x7F, CARD - 10, dtype=np.uint8))
        out += kw + b"= " + val
    out += b"END" + b" " * (CARD - 3)
    return bytes(out)


def padded_len(nbytes: int) -> int:
    return (nbytes + FITS_BLOCK - 1) // FITS_BLOCK * FITS_BLOCK


def fits_image_bytes(rng: np.random.Generator, ny: int, nx: int, mean: float = 1000.0, sigma: float = 30.0,
                     n_sources: int = 10_000, fwhm: float = 6.84, radius: int = 12) -> np.ndarray:
    """Big-endian float32 image (Gaussian noise + Gaussian point sources),
    zero-padded to a multiple of 2880 bytes, as a uint8 array."""
    img = rng.standard_normal(size=(ny, nx), dtype=np.float32)
    img *= np.float32(sigma)
    img += np.float32(mean)
    if n_sources:
        ys = rng.uniform(0, ny, n_sources)
        xs = rng.uniform(0, nx, n_sources)
        amp = 10.0 ** rng.uniform(2.0, 4.0, n_sources)  # log-uniform peak, 100..1e4 ADU
        s = fwhm / 2.3548
        d = np.arange(-radius, radius + 1)
        dy, dx = np.meshgrid(d, d, indexing="ij")
        for lo in range(0, n_sources, 1000):
            hi = min(n_sources, lo + 1000)
            cy = np.floor(ys[lo:hi])[:, None, None] + dy
            cx = np.floor(xs[lo:hi])[:, None, None] + dx
            r2 = (cy + 0.5 - ys[lo:hi, None, None]) ** 2 + (cx + 0.5 - xs[lo:hi, None, None]) ** 2
            val = (amp[lo:hi, None, None] * np.exp(-r2 / (2 * s * s))).astype(np.float32)
            ok = (cy >= 0) & (cy < ny) & (cx >= 0) & (cx < nx)
            np.add.at(img, (cy[ok].astype(np.int64), cx[ok].astype(np.int64)), val[ok])
    raw = ny * nx * 4
    out = np.zeros(padded_len(raw), dtype=np.uint8)
    out[:raw].view(">f4")[:] = img.reshape(-1)
    return out


def fits_file(rng: np.random.Generator, ny: int, nx: int, bitpix: int = -32, n_sources: int = 20) -> bytes:
    """A complete single-HDU FITS image file: a primary header with the
    mandatory keywords, a simple tangent-plane WCS, OBJECT / EXPTIME / DATE-OBS
    cards and a comment, then the big-endian pixels (Gaussian sky noise with
    point sources, cast to BITPIX) zero-padded to a multiple of 2880 bytes.
    The stand-in for the paper's 256x256 float32 test file with
    representative WCS metadata."""
    def card(text: str) -> str:
        return text.ljust(CARD)

    def kv(name: str, value: str) -> str:
        return card(name.ljust(8) + "= " + value)

    def num(name: str, v) -> str:
        return kv(name, str(v).rjust(20))

    def sval(name: str, v: str) -> str:
        return kv(name, "'" + v.ljust(8) + "'")

    cards = [kv("SIMPLE", "T".rjust(20)), num("BITPIX", bitpix), num("NAXIS", 2), num("NAXIS1", nx),
             num("NAXIS2", ny), sval("CTYPE1", "RA---TAN"), sval("CTYPE2", "DEC--TAN"),
             num("CRPIX1", f"{nx / 2 + 0.5:.1f}"), num("CRPIX2", f"{ny / 2 + 0.5:.1f}"),
             num("CRVAL1", f"{rng.uniform(0, 360):.6f}"), num("CRVAL2", f"{rng.uniform(-90, 90):.6f}"),
             num("CDELT1", "-0.000138889"), num("CDELT2", "0.000138889"), sval("OBJECT", "SYNTH_FIELD"),
             num("EXPTIME", f"{rng.uniform(10, 600):.1f}"), sval("DATE-OBS", "2025-01-15T03:12:45"),
             card("COMMENT   synthetic sky image: Gaussian noise and point sources"), card("END")]
    header = "".join(cards).encode("ascii")
    header += b" " * ((-len(header)) % FITS_BLOCK)
    img = fits_image_bytes(rng, ny, nx, n_sources=n_sources)[:ny * nx * 4].view(">f4").astype(np.float64)
    dt = {8: ">u1", 16: ">i2", 32: ">i4", 64: ">i8", -32: ">f4", -64: ">f8"}[bitpix]
    if bitpix > 0:
        hi = {8: 255, 16: 32767, 32: 2**31 - 1, 64: 2**62}[bitpix]
        img = np.clip(np.rint(img), 0, hi)
    data = img.astype(dt).tobytes()
    data += bytes((-len(data)) % FITS_BLOCK)
    return header + data


@dataclass
class Message:
    key: bytes
    iv: bytes
    aad: np.ndarray
    data: np.ndarray  # plaintext (encrypt) or ciphertext source
    op: int = 0       # 0 encrypt, 1 decrypt-verify


# ------------------------------------------------------------------ configs

def config1(seed: int = 2602) -> Message:
    """AES-128-GCM of one 1 MiB message of uniform random bytes, 16-byte AAD."""
    r = rng_for(seed, 1)
    key = random_bytes(r, 16).tobytes()
    iv = random_bytes(r, 12).tobytes()
    aad = random_bytes(r, 16)
    pt = random_bytes(r, 1 << 20)
    return Message(key, iv, aad, pt)


def config2(seed: int = 2602, ny: int = 16384, nx: int = 16384, n_sources: int = 10_000) -> Message:
    """AES-256-GCM of one FITS-shaped buffer: 16384x16384 float32 (1 GiB)
    padded to 1,073,744,640 bytes, AAD = a 2880-byte header."""
    r = rng_for(seed, 2)
    key = random_bytes(r, 32).tobytes()
    iv = random_bytes(r, 12).tobytes()
    aad = np.frombuffer(fits_header(r), dtype=np.uint8).copy()
    pt = fits_image_bytes(rng_for(seed, 2, 1), ny, nx, n_sources=n_sources)
    return Message(key, iv, aad, pt)


def lognormal_lengths(rng: np.random.Generator, n: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    v = rng.lognormal(mean=np.log(median), sigma=sigma, size=n)
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


@dataclass
class BatchSpec:
    lengths: np.ndarray
    key_lens: np.ndarray
    aad_lens: np.ndarray
    keys: List[bytes] = field(default_factory=list)
    ivs: List[bytes] = field(default_factory=list)
    seed: int = 0


def config3_spec(seed: int = 2602, n_msgs: int = 4096, median: float = float(1 << 20),
                 lo: int = 4096, hi: int = 64 << 20, max_aad: int = 4096) -> BatchSpec:
    """Batched uneven messages: lognormal lengths (median 1 MiB, sigma
    sqrt(2 ln 2) so the mean is 2 MiB), clipped to [4 KiB, 64 MiB], per-message
    AES-128 or AES-256 key, IV and 0..4 KiB AAD."""
    r = rng_for(seed, 3)
    lengths = lognormal_lengths(r, n_msgs, median, float(np.sqrt(2 * np.log(2))), lo, hi)
    key_lens = np.where(r.integers(0, 2, n_msgs) == 0, 16, 32)
    aad_lens = r.integers(0, max_aad + 1, n_msgs)
    keys = [random_bytes(r, int(k)).tobytes() for k in key_lens]
    ivs = [random_bytes(r, 12).tobytes() for _ in range(n_msgs)]
    return BatchSpec(lengths, key_lens, aad_lens, keys, ivs, seed)


def batch_payload(spec: BatchSpec, i: int, aad: bool = False) -> np.ndarray:
    """Bytes of message i's payload (or AAD), drawn from its own stream."""
    r = rng_for(spec.seed, 3, 1 + int(aad), i)
    n = int(spec.aad_lens[i] if aad else spec.lengths[i])
    return random_bytes(r, n)


def tamper_plan(seed: int, n_files: int, frac: float = 0.05, tag_prob: float = 0.5):
    """Which files get one flipped bit, and where: exactly round(frac*n)
    files; each flips one bit of the tag (probability tag_prob) or of a
    uniformly chosen ciphertext byte.  Returns {file: ("tag"|"ct", bit_or_byte, bit)}."""
    r = rng_for(seed, 4, 99)
    k = int(round(frac * n_files))
    files = r.choice(n_files, size=k, replace=False)
    plan = {}
    for f in sorted(int(x) for x in files):
        where = "tag" if r.random() < tag_prob else "ct"
        plan[f] = (where, float(r.random()), int(r.integers(0, 8)))
    return plan


def config4_keys(seed: int = 2602, n_files: int = 1024):
    r = rng_for(seed, 4)
    keys = [random_bytes(r, 32).tobytes() for _ in range(n_files)]
    ivs = [random_bytes(r, 12).tobytes() for _ in range(n_files)]
    return keys, ivs


def serving_requests(seed: int, n: int, qps: float, median: float = float(4 << 20),
                     lo: int = 16 << 10, hi: int = 1 << 30, n_keys: int = 1024):
    """Poisson arrivals at `qps`, 50/50 encrypt / decrypt-verify, lognormal
    sizes (median 4 MiB, +-3 sigma spanning 16 KiB..1 GiB) rounded up to a
    2880 multiple, keys uniform over the resident key table."""
    r = rng_for(seed, 5)
    gaps = r.exponential(1.0 / qps, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = lognormal_lengths(r, n, median, float(np.log(2 ** 16) / 6), lo, hi)
    sizes = (sizes + FITS_BLOCK - 1) // FITS_BLOCK * FITS_BLOCK
    ops = r.integers(0, 2, n)
    keys = r.integers(0, n_keys, n)
    return arrivals, sizes, ops, keys


def serving_key_table(seed: int, n_keys: int = 1024):
    """Resident key table: half AES-128, half AES-256."""
    r = rng_for(seed, 5, 1)
    return [random_bytes(r, 16 if i % 2 == 0 else 32).tobytes() for i in range(n_keys)]


def fits_noise_bytes(rng: np.random.Generator, nbytes: int, mean: float = 1000.0, sigma: float = 30.0) -> np.ndarray:
    """`nbytes` (a multiple of 4) of big-endian float32 Gaussian sky noise,
    the pixel content of a FITS-shaped request without point sources."""
    assert nbytes % 4 == 0
    img = rng.standard_normal(size=nbytes // 4, dtype=np.float32)
    img *= np.float32(sigma)
    img += np.float32(mean)
    return img.astype(">f4").view(np.uint8)


@dataclass
class ServingCase:
    op: int            # 0 encrypt, 1 decrypt-verify
    key_index: int     # index into serving_key_table
    iv: bytes
    size: int          # payload bytes (a multiple of 2880)
    tamper: Optional[tuple] = None  # decrypt only: ("tag"|"ct", fraction, bit)


def serving_parity_spec(seed: int = 2602, n: int = 48, big: int = 256 << 20, cap: int = 96 << 20,
                        n_keys: int = 1024, tamper_frac: float = 0.2) -> List[ServingCase]:
    """Requests drawn from the serving workload's distribution (lognormal
    sizes, median 4 MiB, sigma ln(2^16)/6, clipped to [16 KiB, 1 GiB] and
    rounded up to 2880 multiples; 50/50 encrypt / decrypt-verify; keys uniform
    over the resident table), bounded for a parity test: request 0 is an
    encrypt and request 1 a decrypt-verify of at least `big` bytes, the
    others are capped at `cap` bytes; about `tamper_frac` of the decrypts
    carry one flipped tag or ciphertext bit."""
    r = rng_for(seed, 5, 7)
    sizes = lognormal_lengths(r, n, float(4 << 20), float(np.log(2 ** 16) / 6), 16 << 10, 1 << 30)
    sizes = np.minimum(sizes, cap)
    big_pad = (big + FITS_BLOCK - 1) // FITS_BLOCK * FITS_BLOCK
    sizes[0] = big_pad
    sizes[1] = big_pad
    sizes = (sizes + FITS_BLOCK - 1) // FITS_BLOCK * FITS_BLOCK
    ops = r.integers(0, 2, n)
    ops[0], ops[1] = 0, 1
    kidx = r.integers(0, n_keys, n)
    cases = []
    for i in range(n):
        iv = random_bytes(r, 12).tobytes()
        tamper = None
        if ops[i] == 1 and (i == 3 or r.random() < tamper_frac):
            tamper = ("tag" if r.random() < 0.5 else "ct", float(r.random()), int(r.integers(0, 8)))
        cases.append(ServingCase(int(ops[i]), int(kidx[i]), iv, int(sizes[i]), tamper))
    # request 3 is a tampered decrypt whenever it is a decrypt; make sure at least one exists
    if not any(c.tamper for c in cases):
        for c in cases:
            if c.op == 1:
                c.tamper = ("tag", 0.5, 3)
                break
    return cases


def serving_case_data(seed: int, i: int, case: ServingCase):
    """(header AAD, FITS-shaped payload) of serving parity request i."""
    r = rng_for(seed, 5, 8, i)
    aad = np.frombuffer(fits_header(r), dtype=np.uint8).copy()
    return aad, fits_noise_bytes(r, case.size)
