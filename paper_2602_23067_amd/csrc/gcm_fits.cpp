// gcm_fits.cpp -- the paper's authenticated FITS container ("Authenticated
// FITS File Format", "Context Binding via Associated Data (AAD)", "Policy
// Enforcement and Granular Access"): a FITS image becomes a two-HDU file,
//
//   HDU 0 (NAXIS = 0): NONCE_H, NONCE_D, ORIG_BPX/NAX/NA1/NA2, AUTHTAG_H,
//          AUTHTAG_D (HIERARCH cards: the names exceed eight characters) and
//          ENCHDR, the original header encrypted under the header key (base64
//          in a long string continued over CONTINUE cards);
//   HDU 1: a one-row, one-column BINTABLE whose TFORM1 = '<N>B' cell holds
//          the pixel bytes encrypted under the data key,
//
// with AAD_D = NONCE_D || "BITPIX" || "NAXIS" || "NAXIS1" || "NAXIS2" (each
// value in strict ASCII decimal) binding the plaintext structure keywords to
// the pixels.  Both GCM computations run on the GPU through the host
// pipeline; this file only builds and parses FITS cards.
#include <hip/hip_runtime.h>

#include <sys/random.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

namespace {

constexpr size_t kCard = 80;
constexpr size_t kBlock = 2880;

size_t pad_to_block(size_t n) { return (n + kBlock - 1) / kBlock * kBlock; }

// ---------------------------------------------------------------- card writing

std::string card_raw(const std::string &text)
{
    std::string c = text.substr(0, kCard);
    c.resize(kCard, ' ');
    return c;
}

std::string name8(const char *name)
{
    std::string k(name);
    k.resize(8, ' ');
    return k;
}

std::string card_logical(const char *name, bool v)
{
    std::string c = name8(name) + "= ";
    std::string val(20, ' ');
    val[19] = v ? 'T' : 'F';
    return card_raw(c + val);
}

std::string card_int(const char *name, long long v)
{
    std::string s = std::to_string(v);
    std::string val(20 > s.size() ? 20 - s.size() : 0, ' ');
    return card_raw(name8(name) + "= " + val + s);
}

std::string card_str(const char *name, const std::string &v)
{
    std::string s = "'" + v;
    if (v.size() < 8)
        s += std::string(8 - v.size(), ' ');
    s += "'";
    return card_raw(name8(name) + "= " + s);
}

std::string card_hierarch_str(const char *name, const std::string &v)
{
    return card_raw(std::string("HIERARCH ") + name + " = '" + v + "'");
}

const char kB64[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/";

std::string b64_encode(const uint8_t *p, size_t n)
{
    std::string o;
    o.reserve((n + 2) / 3 * 4);
    for (size_t i = 0; i < n; i += 3) {
        const uint32_t b0 = p[i], b1 = i + 1 < n ? p[i + 1] : 0, b2 = i + 2 < n ? p[i + 2] : 0;
        const uint32_t w = (b0 << 16) | (b1 << 8) | b2;
        o += kB64[(w >> 18) & 63];
        o += kB64[(w >> 12) & 63];
        o += i + 1 < n ? kB64[(w >> 6) & 63] : '=';
        o += i + 2 < n ? kB64[w & 63] : '=';
    }
    return o;
}

bool b64_decode(const std::string &s, std::vector<uint8_t> *out)
{
    if (s.size() % 4)
        return false;
    out->clear();
    out->reserve(s.size() / 4 * 3);
    auto val = [](char c) -> int {
        const char *p = std::strchr(kB64, c);
        return (c && p) ? (int)(p - kB64) : -1;
    };
    for (size_t i = 0; i < s.size(); i += 4) {
        int v[4];
        int pad = 0;
        for (int k = 0; k < 4; ++k) {
            if (s[i + k] == '=' && i + 4 == s.size() && k >= 2) {
                v[k] = 0;
                ++pad;
            } else {
                v[k] = val(s[i + k]);
                if (v[k] < 0 || pad)
                    return false;
            }
        }
        const uint32_t w = ((uint32_t)v[0] << 18) | ((uint32_t)v[1] << 12) | ((uint32_t)v[2] << 6) | (uint32_t)v[3];
        out->push_back((uint8_t)(w >> 16));
        if (pad < 2)
            out->push_back((uint8_t)(w >> 8));
        if (pad < 1)
            out->push_back((uint8_t)w);
    }
    return true;
}

std::string hex(const uint8_t *p, size_t n)
{
    static const char d[] = "0123456789ABCDEF";
    std::string o;
    for (size_t i = 0; i < n; ++i) {
        o += d[p[i] >> 4];
        o += d[p[i] & 15];
    }
    return o;
}

bool unhex(const std::string &s, uint8_t *out, size_t n)
{
    if (s.size() != 2 * n)
        return false;
    for (size_t i = 0; i < n; ++i) {
        int v = 0;
        for (int k = 0; k < 2; ++k) {
            const char c = s[2 * i + k];
            const int x = (c >= '0' && c <= '9') ? c - '0' : (c >= 'A' && c <= 'F') ? c - 'A' + 10 : -1;
            if (x < 0)
                return false;
            v = 16 * v + x;
        }
        out[i] = (uint8_t)v;
    }
    return true;
}

// ---------------------------------------------------------------- card reading

struct Header {
    std::vector<std::string> cards;  // up to and including END
    size_t bytes = 0;                // header size on disk (2880 multiple)
};

bool read_header(const uint8_t *p, size_t n, size_t off, Header *h)
{
    h->cards.clear();
    for (size_t q = off; q + kCard <= n; q += kCard) {
        std::string c(reinterpret_cast<const char *>(p + q), kCard);
        h->cards.push_back(c);
        if (c.compare(0, 8, "END     ") == 0) {
            h->bytes = pad_to_block(q + kCard - off);
            return off + h->bytes <= n;
        }
    }
    return false;
}

std::string trim(const std::string &s)
{
    size_t a = s.find_first_not_of(' '), b = s.find_last_not_of(' ');
    return a == std::string::npos ? std::string() : s.substr(a, b - a + 1);
}

// value field of a fixed-format card NAME = value / comment (NULL if absent)
const std::string *find_card(const Header &h, const char *name)
{
    const std::string k = name8(name) + "=";
    for (const std::string &c : h.cards)
        if (c.compare(0, 9, k) == 0)
            return &c;
    return nullptr;
}

bool get_int(const Header &h, const char *name, long long *v)
{
    const std::string *c = find_card(h, name);
    if (!c)
        return false;
    std::string s = c->substr(10);
    const size_t slash = s.find('/');
    if (slash != std::string::npos)
        s = s.substr(0, slash);
    s = trim(s);
    if (s.empty())
        return false;
    char *end = nullptr;
    *v = std::strtoll(s.c_str(), &end, 10);
    return end && *end == 0;
}

// the string between the quotes starting at position `q` of card `c`
bool quoted(const std::string &c, size_t q, std::string *out)
{
    if (q >= c.size() || c[q] != '\'')
        return false;
    out->clear();
    for (size_t i = q + 1; i < c.size(); ++i) {
        if (c[i] == '\'') {
            if (i + 1 < c.size() && c[i + 1] == '\'') {
                *out += '\'';
                ++i;
                continue;
            }
            return true;
        }
        *out += c[i];
    }
    return false;
}

bool get_str(const Header &h, const char *name, std::string *v)
{
    const std::string *c = find_card(h, name);
    if (!c)
        return false;
    const size_t q = c->find('\'', 10);
    if (q == std::string::npos || !quoted(*c, q, v))
        return false;
    *v = trim(*v);
    return true;
}

bool get_hierarch_str(const Header &h, const char *name, std::string *v)
{
    const std::string k = std::string("HIERARCH ") + name + " = ";
    for (const std::string &c : h.cards)
        if (c.compare(0, k.size(), k) == 0)
            return quoted(c, k.size(), v);
    return false;
}

// a long string value continued over CONTINUE cards ('&' before each closing quote)
bool get_long_str(const Header &h, const char *name, std::string *v)
{
    const std::string k = name8(name) + "= ";
    v->clear();
    for (size_t i = 0; i < h.cards.size(); ++i) {
        if (h.cards[i].compare(0, 10, k) != 0)
            continue;
        std::string part;
        if (!quoted(h.cards[i], 10, &part))
            return false;
        for (size_t j = i + 1;; ++j) {
            const bool more = !part.empty() && part.back() == '&';
            if (more)
                part.pop_back();
            *v += part;
            if (!more)
                return true;
            if (j >= h.cards.size() || h.cards[j].compare(0, 10, "CONTINUE  ") != 0 ||
                !quoted(h.cards[j], 10, &part))
                return false;
        }
    }
    return false;
}

struct Structure {
    long long bitpix = 0, naxis = 0, naxis1 = 0, naxis2 = 0;
};

// AAD_D = NONCE_D || strict ASCII decimal of BITPIX, NAXIS, NAXIS1, NAXIS2
std::vector<uint8_t> data_aad(const uint8_t nonce_d[12], const Structure &s)
{
    std::vector<uint8_t> a(nonce_d, nonce_d + 12);
    for (long long v : {s.bitpix, s.naxis, s.naxis1, s.naxis2}) {
        const std::string t = std::to_string(v);
        a.insert(a.end(), t.begin(), t.end());
    }
    return a;
}

uint64_t data_bytes(const Structure &s)
{
    const long long b = s.bitpix < 0 ? -s.bitpix : s.bitpix;
    return (uint64_t)(b / 8) * (uint64_t)s.naxis1 * (uint64_t)s.naxis2;
}

// a 2-D image whose pixel bytes fit the GCM length limit (so no size below overflows)
bool valid_structure(const Structure &s)
{
    const long long b = s.bitpix;
    const bool bp = b == 8 || b == 16 || b == 32 || b == 64 || b == -32 || b == -64;
    if (!bp || s.naxis != 2 || s.naxis1 < 0 || s.naxis2 < 0 || (uint64_t)s.naxis1 > kMaxLen ||
        (uint64_t)s.naxis2 > kMaxLen)
        return false;
    const unsigned __int128 n = (unsigned __int128)(uint64_t)((b < 0 ? -b : b) / 8) * (uint64_t)s.naxis1 *
                                (uint64_t)s.naxis2;
    return n <= kMaxLen;
}

void append_cards(std::vector<uint8_t> *out, const std::vector<std::string> &cards)
{
    const size_t start = out->size();
    for (const std::string &c : cards)
        out->insert(out->end(), c.begin(), c.end());
    out->resize(start + pad_to_block(out->size() - start), ' ');
}

// the result buffer is allocated once at its final size and filled in place
// (payloads are encrypted or decrypted straight into it)
int result_alloc(gcm_fits_result *r, uint64_t bytes)
{
    r->data = static_cast<uint8_t *>(std::malloc(bytes ? bytes : 1));
    if (!r->data)
        return fail(GCM_E_NOMEM, "host allocation of %llu bytes failed", (unsigned long long)bytes);
    r->size = bytes;
    return GCM_OK;
}

std::vector<uint8_t> card_bytes(const std::vector<std::string> &cards)
{
    std::vector<uint8_t> b;
    append_cards(&b, cards);
    return b;
}

int finish(gcm_fits_result *r, int rc)
{
    r->error_code = rc;
    return rc;
}

}  // namespace

extern "C" int gcm_fits_nonce(uint8_t out[12])
{
    GCM_ABI_TRY
        if (!out)
            return fail(GCM_E_ARG, "NULL argument");
        size_t got = 0;
        while (got < 12) {
            const ssize_t k = getrandom(out + got, 12 - got, 0);
            if (k <= 0)
                return fail(GCM_E_ARG, "getrandom failed");
            got += (size_t)k;
        }
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" void gcm_fits_free(gcm_fits_result *r)
{
    GCM_ABI_TRY
        if (r && r->data) {
            std::free(r->data);
            r->data = nullptr;
            r->size = 0;
        }
    GCM_ABI_CATCH_VOID
}

extern "C" int gcm_fits_encrypt(gcm_ctx *ctx, const uint8_t *fits, uint64_t fits_len, const uint8_t *key_h,
                                size_t key_h_len, const uint8_t *key_d, size_t key_d_len, const uint8_t nonce_h[12],
                                const uint8_t nonce_d[12], gcm_fits_result *out)
{
    GCM_ABI_TRY
        if (!out)
            return fail(GCM_E_ARG, "NULL result");
        std::memset(out, 0, sizeof *out);
        if (!ctx || !fits || !key_h || !key_d || !nonce_h || !nonce_d)
            return finish(out, fail(GCM_E_ARG, "NULL argument"));
        Header h;
        if (!read_header(fits, fits_len, 0, &h) || h.cards[0].compare(0, 9, "SIMPLE  =") != 0)
            return finish(out, fail(GCM_E_ARG, "input is not a FITS file with a complete primary header"));
        Structure s;
        if (!get_int(h, "BITPIX", &s.bitpix) || !get_int(h, "NAXIS", &s.naxis) || !get_int(h, "NAXIS1", &s.naxis1) ||
            !get_int(h, "NAXIS2", &s.naxis2) || !valid_structure(s))
            return finish(out, fail(GCM_E_ARG, "primary HDU must be a 2-D image (BITPIX 8/16/32/64/-32/-64)"));
        const uint64_t nd = data_bytes(s);
        if (nd > fits_len || h.bytes > fits_len - nd)
            return finish(out, fail(GCM_E_ARG, "FITS data shorter than NAXIS1 x NAXIS2 x |BITPIX|/8"));

        // header encrypted on the GPU (host pipeline); the HDU 0 cards need its tag
        std::vector<uint8_t> ct_h(h.bytes);
        uint8_t tag_h[16], tag_d[16];
        int rc = gcm_encrypt_host(ctx, key_h, key_h_len, nonce_h, 12, nonce_h, 12, fits, h.bytes, ct_h.data(), tag_h);
        if (rc)
            return finish(out, rc);
        // the HDU 0 and HDU 1 headers have fixed sizes (the tags are fixed-width
        // hex), so the pixels are encrypted straight into their final place
        const std::string enc = b64_encode(ct_h.data(), ct_h.size());
        constexpr size_t kChunk = 64;
        const size_t enc_cards = enc.empty() ? 1 : (enc.size() + kChunk - 1) / kChunk;
        const size_t h0_bytes = pad_to_block((14 + enc_cards) * kCard), h1_bytes = kBlock;
        rc = result_alloc(out, h0_bytes + h1_bytes + pad_to_block(nd));
        if (rc)
            return finish(out, rc);
        uint8_t *blob = out->data + h0_bytes + h1_bytes;
        {
            const std::vector<uint8_t> aad = data_aad(nonce_d, s);
            rc = gcm_encrypt_host(ctx, key_d, key_d_len, nonce_d, 12, aad.data(), aad.size(), fits + h.bytes, nd, blob,
                                  tag_d);
        }
        if (rc) {
            gcm_fits_free(out);
            return finish(out, rc);
        }
        std::memset(blob + nd, 0, pad_to_block(nd) - nd);

        std::vector<std::string> c0 = {card_logical("SIMPLE", true), card_int("BITPIX", 8), card_int("NAXIS", 0),
                                       card_logical("EXTEND", true), card_str("LONGSTRN", "OGIP 1.0"),
                                       card_str("NONCE_H", hex(nonce_h, 12)), card_str("NONCE_D", hex(nonce_d, 12)),
                                       card_int("ORIG_BPX", s.bitpix), card_int("ORIG_NAX", s.naxis),
                                       card_int("ORIG_NA1", s.naxis1), card_int("ORIG_NA2", s.naxis2),
                                       card_hierarch_str("AUTHTAG_H", hex(tag_h, 16)),
                                       card_hierarch_str("AUTHTAG_D", hex(tag_d, 16))};
        for (size_t i = 0; i < enc.size() || i == 0; i += kChunk) {
            const bool last = i + kChunk >= enc.size();
            const std::string part = enc.substr(i, kChunk) + (last ? "" : "&");
            c0.push_back(card_raw((i == 0 ? std::string("ENCHDR  = '") : std::string("CONTINUE  '")) + part + "'"));
        }
        c0.push_back(card_raw("END"));
        std::vector<std::string> c1 = {card_str("XTENSION", "BINTABLE"), card_int("BITPIX", 8), card_int("NAXIS", 2),
                                       card_int("NAXIS1", (long long)nd), card_int("NAXIS2", 1), card_int("PCOUNT", 0),
                                       card_int("GCOUNT", 1), card_int("TFIELDS", 1), card_str("TTYPE1", "BLOB"),
                                       card_str("TFORM1", std::to_string(nd) + "B"), card_raw("END")};
        const std::vector<uint8_t> b0 = card_bytes(c0), b1 = card_bytes(c1);
        if (b0.size() != h0_bytes || b1.size() != h1_bytes) {  // the fixed layout above must hold
            gcm_fits_free(out);
            return finish(out, fail(GCM_E_ARG, "internal: container header sizes %zu/%zu", b0.size(), b1.size()));
        }
        std::memcpy(out->data, b0.data(), h0_bytes);
        std::memcpy(out->data + h0_bytes, b1.data(), h1_bytes);
        out->warning_code = 0;
        return finish(out, GCM_OK);
    GCM_ABI_CATCH
}

extern "C" int gcm_fits_decrypt(gcm_ctx *ctx, const uint8_t *container, uint64_t len, const uint8_t *key_h,
                                size_t key_h_len, const uint8_t *key_d, size_t key_d_len, gcm_fits_result *out)
{
    GCM_ABI_TRY
        if (!out)
            return fail(GCM_E_ARG, "NULL result");
        std::memset(out, 0, sizeof *out);
        if (!ctx || !container)
            return finish(out, fail(GCM_E_ARG, "NULL argument"));
        Header h0, h1;
        Structure s;
        std::string nh, nd_hex, th, td, enc;
        uint8_t nonce_h[12], nonce_d[12], tag_h[16], tag_d[16];
        if (!read_header(container, len, 0, &h0) || !read_header(container, len, h0.bytes, &h1) ||
            !get_int(h0, "ORIG_BPX", &s.bitpix) || !get_int(h0, "ORIG_NAX", &s.naxis) ||
            !get_int(h0, "ORIG_NA1", &s.naxis1) || !get_int(h0, "ORIG_NA2", &s.naxis2) || !valid_structure(s) ||
            !get_str(h0, "NONCE_H", &nh) || !get_str(h0, "NONCE_D", &nd_hex) || !unhex(nh, nonce_h, 12) ||
            !unhex(nd_hex, nonce_d, 12) || !get_hierarch_str(h0, "AUTHTAG_H", &th) ||
            !get_hierarch_str(h0, "AUTHTAG_D", &td) || !unhex(th, tag_h, 16) || !unhex(td, tag_d, 16) ||
            !get_long_str(h0, "ENCHDR", &enc))
            return finish(out, fail(GCM_E_ARG, "not an authenticated FITS container"));
        // the blob: N bytes as the BINTABLE declares them
        long long nblob = -1;
        std::string tform;
        if (!get_int(h1, "NAXIS1", &nblob) || nblob < 0 || (uint64_t)nblob > len || !get_str(h1, "TFORM1", &tform) ||
            tform != std::to_string(nblob) + "B" || h0.bytes + h1.bytes > len - (uint64_t)nblob)
            return finish(out, fail(GCM_E_ARG, "container blob is not a %lld-byte TFORM1 cell", nblob));
        std::vector<uint8_t> ct_h;
        if (!b64_decode(enc, &ct_h) || ct_h.empty() || ct_h.size() % kBlock)
            return finish(out, fail(GCM_E_ARG, "ENCHDR is not a base64 FITS header"));
        const uint8_t *ct_d = container + h0.bytes + h1.bytes;

        int warn = 0;
        // header: the authenticated original, else a minimal header from ORIG_*;
        // the output pixels take the shape of whichever header is returned
        std::vector<uint8_t> header(ct_h.size());
        int ok_h = 0;
        if (key_h) {
            int rc = gcm_decrypt_verify_host(ctx, key_h, key_h_len, nonce_h, 12, nonce_h, 12, ct_h.data(), ct_h.size(),
                                             tag_h, header.data(), &ok_h);
            if (rc && rc != GCM_E_KEYLEN)
                return finish(out, rc);
            if (rc == GCM_E_KEYLEN)
                ok_h = 0;
        }
        Structure so = s;
        if (ok_h) {
            Header ho;
            if (!read_header(header.data(), header.size(), 0, &ho) || !get_int(ho, "BITPIX", &so.bitpix) ||
                !get_int(ho, "NAXIS", &so.naxis) || !get_int(ho, "NAXIS1", &so.naxis1) ||
                !get_int(ho, "NAXIS2", &so.naxis2) || !valid_structure(so))
                return finish(out, fail(GCM_E_ARG, "authenticated header is not a 2-D image header"));
            header.resize(ho.bytes);
        } else {
            header.clear();
            append_cards(&header, {card_logical("SIMPLE", true), card_int("BITPIX", s.bitpix), card_int("NAXIS", s.naxis),
                                   card_int("NAXIS1", s.naxis1), card_int("NAXIS2", s.naxis2), card_raw("END")});
            warn |= 1;
        }
        const uint64_t nout = data_bytes(so);
        const size_t d0 = header.size();
        int rc = result_alloc(out, d0 + pad_to_block(nout));
        if (rc)
            return finish(out, rc);
        std::memcpy(out->data, header.data(), d0);
        uint8_t *pix = out->data + d0;
        // pixels: authenticated plaintext, else zeros (payload suppression); a blob
        // whose size differs from the output shape cannot authenticate
        int ok_d = 0;
        if (key_d && (uint64_t)nblob == nout) {
            const std::vector<uint8_t> aad = data_aad(nonce_d, s);
            rc = gcm_decrypt_verify_host(ctx, key_d, key_d_len, nonce_d, 12, aad.data(), aad.size(), ct_d, nout, tag_d,
                                         pix, &ok_d);
            if (rc && rc != GCM_E_KEYLEN) {
                gcm_fits_free(out);
                return finish(out, rc);
            }
            if (rc == GCM_E_KEYLEN)
                ok_d = 0;
        }
        if (!ok_d) {
            std::memset(pix, 0, nout);
            warn |= 2;
        }
        std::memset(pix + nout, 0, pad_to_block(nout) - nout);
        out->warning_code = warn;
        return finish(out, GCM_OK);
    GCM_ABI_CATCH
}
