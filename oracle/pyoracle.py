"""ctypes wrapper of the CPU oracle.  TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  The product library never does.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("ORC_LIB")   # a prebuilt oracle (the sanitizer build)
        if not path:
            if not os.path.exists(_build.OUT):
                _build.build()
            path = _build.OUT
        _LIB = C.CDLL(path)
        _declare(_LIB)
    return _LIB


class OrcLayout(C.Structure):
    _fields_ = [(n, C.c_int) for n in
                ("kind", "bs", "c", "h", "w", "M", "S", "m", "bsg", "cpc", "nbg", "ncg",
                 "rep", "dil", "level", "d", "nfeat")] + [("scale", C.c_double),
                                                          ("pos", C.POINTER(C.c_int))]


LAYOUT_FIELDS = ("kind", "bs", "c", "h", "w", "M", "S", "m", "bsg", "cpc", "nbg", "ncg",
                 "rep", "dil", "level", "d", "nfeat", "scale")
COUNT_FIELDS = ("inner_rot", "outer_rot", "other_rot", "ks", "modup", "moddown",
                "pmult", "smult", "rescale", "relin")

u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def _declare(L):
    vp, i, d, u = C.c_void_p, C.c_int, C.c_double, C.c_uint64
    sig = {
        "orc_last_error": (C.c_char_p, []),
        "orc_new": (vp, [i, i, i, i, i, i, d, u]),
        "orc_free": (None, [vp]),
        "orc_primes": (i, [vp, u64p]),
        "orc_psi": (None, [vp, u64p]),
        "orc_secret": (None, [vp, i64p]),
        "orc_is_prime": (i, [u]),
        "orc_rng": (u, [u, u, u]),
        "orc_ternary": (i, [u, u, u]),
        "orc_gauss": (i, [u, u, u]),
        "orc_uniform": (u, [u, u, u, u]),
        "orc_gauss_cdt": (None, [u64p]),
        "orc_polymul": (i, [vp, i, u64p, u64p, u64p, i]),
        "orc_ntt": (i, [vp, i, u64p, i]),
        "orc_automorph": (i, [vp, i, u64p, u, u64p]),
        "orc_galois": (u, [vp, C.c_int64]),
        "orc_encode_int": (i, [vp, f64p, vp, d, i64p, i]),
        "orc_encode": (i, [vp, f64p, vp, d, i, u64p]),
        "orc_decode": (i, [vp, u64p, d, f64p, f64p]),
        "orc_encrypt": (i, [vp, u64p, i, d, u, u, u64p]),
        "orc_decrypt": (i, [vp, u64p, i, u64p]),
        "orc_switch_key": (i, [vp, u, u64p]),
        "orc_mod_up": (i, [vp, u64p, i, u64p]),
        "orc_mod_down": (i, [vp, u64p, i, u64p]),
        "orc_mod_down_rescale": (i, [vp, u64p, i, u64p]),
        "orc_rotate": (i, [vp, u64p, i, i64p, i, u64p]),
        "orc_rotate_sum": (i, [vp, vp, u64p, i64p, i, i, u64p]),
        "orc_rescale": (i, [vp, u64p, i, u64p]),
        "orc_square_relin": (i, [vp, u64p, i, u64p]),
        "orc_rot_total_formula": (d, [d, d, d, d, d, d]),
        "orc_rot_inner_formula_eq": (d, [d, d, d, d, d]),
        "orc_optimal_S": (d, [d, d, d, d, d]),
        "orc_plan_layout": (i, [vp, i, i, i, i, i, i, i, C.POINTER(OrcLayout)]),
        "orc_fragment_layout": (i, [vp, i, i, i, i, i, C.POINTER(OrcLayout)]),
        "orc_token_layout": (i, [vp, i, i, i, C.POINTER(OrcLayout)]),
        "orc_element_slots": (i, [C.POINTER(OrcLayout), i, i, i, i, C.POINTER(C.c_int), i]),
        "orc_encrypt_tensor": (vp, [vp, C.POINTER(OrcLayout), f64p, u]),
        "orc_encode_tensor": (i, [vp, C.POINTER(OrcLayout), f64p, u64p]),
        "orc_batch_from": (vp, [vp, C.POINTER(OrcLayout), u64p]),
        "orc_batch_free": (None, [vp]),
        "orc_batch_layout": (None, [vp, C.POINTER(OrcLayout)]),
        "orc_batch_data": (i, [vp, vp, u64p]),
        "orc_decrypt_tensor": (i, [vp, vp, f64p]),
        "orc_conv2d": (vp, [vp, vp, f64p, i, i, i, i, i, C.c_longlong, i, C.POINTER(OrcLayout), vp, vp, i, i,
                            C.POINTER(C.c_long)]),
        "orc_avgpool2": (vp, [vp, vp, i, C.POINTER(C.c_long)]),
        "orc_pq_roundtrip": (i, [vp, u64p, i, vp, i, i, u64p]),
        "orc_square": (vp, [vp, vp, C.POINTER(C.c_long)]),
        "orc_poly_act": (vp, [vp, vp, f64p, i, C.POINTER(C.c_long)]),
        "orc_compress": (vp, [vp, vp, C.POINTER(OrcLayout), i, C.POINTER(C.c_long)]),
        "orc_fc": (vp, [vp, vp, f64p, i, vp, vp, i, C.POINTER(C.c_long)]),
        "orc_weight_code": (C.c_int64, [d, d]),
        "orc_time_ops": (i, [vp, i, i, i, f64p]),
        "orc_split_scale": (None, [d, C.POINTER(d), C.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc is None or (isinstance(rc, int) and rc < 0):
        raise OracleError(lib().orc_last_error().decode())
    return rc


def layout_n_ct(L):
    """Ciphertexts of a layout: S^2 per (batch group, channel group) for
    fragments, S per chunk of a token group, one per group for vectors."""
    if L["kind"] == 0:
        return L["nbg"] * L["ncg"] * L["S"] ** 2
    if L["kind"] == 2:
        return L["nbg"] * L["S"] * L["ncg"]
    return L["nbg"]


def layout_to_dict(lay, pos=None):
    d = {k: getattr(lay, k) for k in LAYOUT_FIELDS}
    d["pos"] = list(pos[:lay.nfeat]) if (pos is not None and lay.kind == 1) else None
    return d


def dict_to_layout(d):
    lay = OrcLayout()
    for k in LAYOUT_FIELDS:
        setattr(lay, k, d[k])
    buf = None
    if d.get("pos") is not None:
        buf = (C.c_int * max(1, len(d["pos"])))(*d["pos"])
        lay.pos = C.cast(buf, C.POINTER(C.c_int))
    else:
        lay.pos = C.POINTER(C.c_int)()
    return lay, buf


class Batch:
    """Oracle-side ciphertext batch (layout + ciphertexts)."""

    def __init__(self, orc, handle):
        self.orc, self.h = orc, handle

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.orc_batch_free(self.h)
            self.h = None

    def layout(self):
        lay = OrcLayout()
        buf = (C.c_int * self.orc.ns)()
        lay.pos = C.cast(buf, C.POINTER(C.c_int))
        lib().orc_batch_layout(self.h, C.byref(lay))
        return layout_to_dict(lay, buf)

    def data(self):
        L = self.layout()
        out = np.zeros((layout_n_ct(L), 2, L["level"] + 1, self.orc.N), np.uint64)
        lib().orc_batch_data(self.orc.h, self.h, out)
        return out


class Oracle:
    """One oracle context: parameters, primes, secret key, key cache."""

    def __init__(self, logN, nq, qbits, np_, pbits, dnum, log2scale, seed):
        self.h = lib().orc_new(logN, nq, qbits, np_, pbits, dnum, log2scale, seed)
        if not self.h:
            raise OracleError(lib().orc_last_error().decode())
        self.logN, self.N, self.ns = logN, 1 << logN, 1 << (logN - 1)
        self.nq, self.np, self.dnum, self.log2scale = nq, np_, dnum, log2scale
        self.alpha = (nq + dnum - 1) // dnum
        self.L = nq - 1

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.orc_free(self.h)
            self.h = None

    # ------------------------------------------------------------ core
    def primes(self):
        out = np.zeros(self.nq + self.np, np.uint64)
        lib().orc_primes(self.h, out)
        return [int(x) for x in out]

    def psi(self):
        out = np.zeros(self.nq + self.np, np.uint64)
        lib().orc_psi(self.h, out)
        return [int(x) for x in out]

    def secret(self):
        out = np.zeros(self.N, np.int64)
        lib().orc_secret(self.h, out)
        return out

    def polymul(self, pidx, a, b, schoolbook=False):
        out = np.zeros(self.N, np.uint64)
        _check(lib().orc_polymul(self.h, pidx, np.ascontiguousarray(a, np.uint64),
                                 np.ascontiguousarray(b, np.uint64), out, int(schoolbook)))
        return out

    def ntt(self, pidx, a, inverse=False):
        x = np.array(a, np.uint64)
        _check(lib().orc_ntt(self.h, pidx, x, int(inverse)))
        return x

    def automorph(self, pidx, a, g):
        out = np.zeros(self.N, np.uint64)
        _check(lib().orc_automorph(self.h, pidx, np.ascontiguousarray(a, np.uint64), g, out))
        return out

    def galois(self, shift):
        return int(lib().orc_galois(self.h, shift))

    def encode_int(self, re, im=None, scale=None, direct=False):
        scale = 2.0 ** self.log2scale if scale is None else scale
        out = np.zeros(self.N, np.int64)
        imarr = None if im is None else np.ascontiguousarray(im, np.float64)
        _check(lib().orc_encode_int(self.h, np.ascontiguousarray(re, np.float64),
                                    None if imarr is None else imarr.ctypes.data, scale, out,
                                    int(direct)))
        return out

    def encode(self, re, im=None, scale=None, level=None):
        scale = 2.0 ** self.log2scale if scale is None else scale
        level = self.L if level is None else level
        out = np.zeros((level + 1, self.N), np.uint64)
        imarr = None if im is None else np.ascontiguousarray(im, np.float64)
        _check(lib().orc_encode(self.h, np.ascontiguousarray(re, np.float64),
                                None if imarr is None else imarr.ctypes.data, scale, level, out))
        return out

    def decode(self, limb0, scale=None):
        scale = 2.0 ** self.log2scale if scale is None else scale
        re = np.zeros(self.ns)
        im = np.zeros(self.ns)
        _check(lib().orc_decode(self.h, np.ascontiguousarray(limb0, np.uint64), scale, re, im))
        return re + 1j * im

    def encrypt(self, pt, level, scale, seed, ct_index=0):
        out = np.zeros((2, level + 1, self.N), np.uint64)
        _check(lib().orc_encrypt(self.h, np.ascontiguousarray(pt, np.uint64), level, scale, seed,
                                 ct_index, out))
        return out

    def decrypt(self, ct):
        level = ct.shape[1] - 1
        out = np.zeros((level + 1, self.N), np.uint64)
        _check(lib().orc_decrypt(self.h, np.ascontiguousarray(ct, np.uint64), level, out))
        return out

    def switch_key(self, keyid):
        ndig = (self.nq + self.alpha - 1) // self.alpha
        out = np.zeros((ndig, 2, self.nq + self.np, self.N), np.uint64)
        _check(lib().orc_switch_key(self.h, keyid, out))
        return out

    def mod_up(self, d, level):
        beta = (level + 1 + self.alpha - 1) // self.alpha
        out = np.zeros((beta, level + 1 + self.np, self.N), np.uint64)
        _check(lib().orc_mod_up(self.h, np.ascontiguousarray(d, np.uint64), level, out))
        return out

    def mod_down(self, a, level):
        out = np.zeros((level + 1, self.N), np.uint64)
        _check(lib().orc_mod_down(self.h, np.ascontiguousarray(a, np.uint64), level, out))
        return out

    def mod_down_rescale(self, a, level):
        out = np.zeros((level, self.N), np.uint64)
        _check(lib().orc_mod_down_rescale(self.h, np.ascontiguousarray(a, np.uint64), level, out))
        return out

    def rotate(self, ct, shifts):
        level = ct.shape[1] - 1
        out = np.zeros((len(shifts), 2, level + 1, self.N), np.uint64)
        _check(lib().orc_rotate(self.h, np.ascontiguousarray(ct, np.uint64), level,
                                np.array(shifts, np.int64), len(shifts), out))
        return out

    def pq_roundtrip(self, ct, shifts=(), lift=False):
        """ModDown of the extended-basis rotations (or of the lift P x)."""
        level = ct.shape[1] - 1
        out = np.zeros((max(1, len(shifts)), 2, level + 1, self.N), np.uint64)
        sh = np.array(list(shifts) or [0], np.int64)
        _check(lib().orc_pq_roundtrip(self.h, np.ascontiguousarray(ct, np.uint64), level, sh.ctypes.data,
                                      len(shifts), int(lift), out))
        return out[0] if lift else out

    def rotate_sum(self, z0, zs, shifts):
        level = zs.shape[2] - 1
        out = np.zeros((2, level + 1, self.N), np.uint64)
        z0p = None if z0 is None else np.ascontiguousarray(z0, np.uint64)
        _check(lib().orc_rotate_sum(self.h, None if z0p is None else z0p.ctypes.data,
                                    np.ascontiguousarray(zs, np.uint64), np.array(shifts, np.int64),
                                    len(shifts), level, out))
        return out

    def rescale(self, ct):
        level = ct.shape[1] - 1
        out = np.zeros((2, level, self.N), np.uint64)
        _check(lib().orc_rescale(self.h, np.ascontiguousarray(ct, np.uint64), level, out))
        return out

    def square_relin(self, ct):
        level = ct.shape[1] - 1
        out = np.zeros((2, level + 1, self.N), np.uint64)
        _check(lib().orc_square_relin(self.h, np.ascontiguousarray(ct, np.uint64), level, out))
        return out

    # ------------------------------------------------------------ method
    def plan_layout(self, bs, c, h, w, k, cout, s_override=0):
        lay = OrcLayout()
        lay.pos = C.POINTER(C.c_int)()
        _check(lib().orc_plan_layout(self.h, bs, c, h, w, k, cout, s_override, C.byref(lay)))
        return layout_to_dict(lay)

    def fragment_layout(self, bs, c, h, w, S):
        lay = OrcLayout()
        lay.pos = C.POINTER(C.c_int)()
        _check(lib().orc_fragment_layout(self.h, bs, c, h, w, S, C.byref(lay)))
        return layout_to_dict(lay)

    def token_layout(self, n, E, S):
        """Token embeddings of E features, n tokens, split into S fragments
        (feature e in fragment e mod S at position e div S)."""
        lay = OrcLayout()
        _check(lib().orc_token_layout(self.h, n, E, S, C.byref(lay)))
        return layout_to_dict(lay)

    def element_slots(self, layout, b, ch, hh, ww):
        lay, keep = dict_to_layout(layout)
        out = (C.c_int * 2048)()
        n = _check(lib().orc_element_slots(C.byref(lay), b, ch, hh, ww, out, 1024))
        return [(out[2 * i], out[2 * i + 1]) for i in range(n)]

    def encode_tensor(self, layout, x):
        lay, keep = dict_to_layout(layout)
        out = np.zeros((layout_n_ct(layout), layout["level"] + 1, self.N), np.uint64)
        _check(lib().orc_encode_tensor(self.h, C.byref(lay), np.ascontiguousarray(x, np.float64), out))
        return out

    def encrypt_tensor(self, layout, x, seed):
        lay, keep = dict_to_layout(layout)
        h = lib().orc_encrypt_tensor(self.h, C.byref(lay), np.ascontiguousarray(x, np.float64), seed)
        return Batch(self, _check(h))

    def batch(self, layout, data):
        lay, keep = dict_to_layout(layout)
        h = lib().orc_batch_from(self.h, C.byref(lay), np.ascontiguousarray(data, np.uint64))
        return Batch(self, _check(h))

    def decrypt_slots(self, batch):
        """Real parts of the decoded slots of every ciphertext of a batch."""
        scale = batch.layout()["scale"]
        return [self.decode(self.decrypt(ct)[0], scale).real for ct in batch.data()]

    def decrypt_tensor(self, batch):
        L = batch.layout()
        x = np.zeros((L["bs"], L["c"], L["h"], L["w"]))
        _check(lib().orc_decrypt_tensor(self.h, batch.h, x))
        return x

    def _op(self, fn, *args):
        cnt = (C.c_long * 10)()
        h = fn(self.h, *args, cnt)
        if not h:
            raise OracleError(lib().orc_last_error().decode())
        return Batch(self, h), dict(zip(COUNT_FIELDS, list(cnt)))

    def conv2d(self, batch, w, stride=1, pad=0, groups=1, pt_budget=1 << 30, hoist=0, target=None, bias=None,
               outputs=None, baby=1):
        """hoist=1: the linear combination is taken in the extended basis Q_l U P
        and each combined ciphertext is moved down once.  target: a layout dict
        of the output tensor the result is written into (the repack fused with
        the convolution); bias: cout values added after the rescale; outputs:
        compute only these output ciphertexts (their input cone), returned as
        an array [len(outputs)][2][level+1][N] instead of a batch; baby: the
        baby step n1 of the outer rotations' baby-step giant-step form (1: the
        plain form, C' - 1 rotations per output)."""
        w = np.ascontiguousarray(w, np.float64)
        t, keep = (None, None) if target is None else dict_to_layout(target)
        b = None if bias is None else np.ascontiguousarray(bias, np.float64)
        outs = None if outputs is None else np.ascontiguousarray(outputs, np.int32)
        res = self._op(lib().orc_conv2d, batch.h, w, w.shape[0], w.shape[2], stride, pad, groups, pt_budget,
                       hoist, None if t is None else C.byref(t), None if b is None else b.ctypes.data,
                       None if outs is None else outs.ctypes.data, 0 if outs is None else len(outs), baby)
        if outs is None:
            return res
        bat, cnt = res
        lvl = bat.layout()["level"]
        data = np.zeros((len(outs), 2, lvl + 1, self.N), np.uint64)
        _check(lib().orc_batch_data(self.h, bat.h, data))   # writes the len(outputs) ciphertexts
        return data, cnt

    def avgpool2(self, batch, hoist=0):
        return self._op(lib().orc_avgpool2, batch.h, hoist)

    def square(self, batch):
        return self._op(lib().orc_square, batch.h)

    def poly_act(self, batch, coeffs):
        c = np.ascontiguousarray(coeffs, np.float64)
        return self._op(lib().orc_poly_act, batch.h, c, len(c))

    def compress(self, batch, target=None, hoist=0):
        """target: a layout dict of the same tensor (None: one VECTOR ciphertext
        per batch group, placed by first fit)."""
        t, keep = (None, None) if target is None else dict_to_layout(target)
        return self._op(lib().orc_compress, batch.h, None if t is None else C.byref(t), hoist)

    def fc(self, batch, w, bias=None, outputs=None):
        """outputs (token layouts): compute only these output ciphertexts,
        returned as an array [len(outputs)][2][level+1][N] instead of a batch."""
        w = np.ascontiguousarray(w, np.float64)
        b = None if bias is None else np.ascontiguousarray(bias, np.float64)
        outs = None if outputs is None else np.ascontiguousarray(outputs, np.int32)
        res = self._op(lib().orc_fc, batch.h, w, w.shape[0], None if b is None else b.ctypes.data,
                       None if outs is None else outs.ctypes.data, 0 if outs is None else len(outs))
        if outs is None:
            return res
        bat, cnt = res
        lvl = bat.layout()["level"]
        data = np.zeros((len(outs), 2, lvl + 1, self.N), np.uint64)
        _check(lib().orc_batch_data(self.h, bat.h, data))   # writes the len(outputs) ciphertexts
        return data, cnt


def time_ops(orc, level, threads=1, reps=1):
    """Seconds per operation of the oracle's primitives at `level` with
    `threads` threads (each on its own ciphertext): modup_rot (ModUp and one
    hoisted rotation), rot (each further hoisted rotation), pmult, smult,
    rescale, square_relin."""
    out = np.zeros(6)
    _check(lib().orc_time_ops(orc.h, level, threads, reps, out))
    return dict(zip(["modup_rot", "rot", "pmult", "smult", "rescale", "square_relin"], out.tolist()))


def rot_total_formula(BS, Nin, Nout, K, S, alpha):
    return lib().orc_rot_total_formula(BS, Nin, Nout, K, S, alpha)


def rot_inner_formula_eq(Nin, K, S, M, alpha):
    return lib().orc_rot_inner_formula_eq(Nin, K, S, M, alpha)


def optimal_S(K, Nin, Nout, alpha, BS):
    return lib().orc_optimal_S(K, Nin, Nout, alpha, BS)


def weight_code(w, scale):
    return int(lib().orc_weight_code(w, scale))


def split_scale(T):
    dw, dm = C.c_double(), C.c_double()
    lib().orc_split_scale(T, C.byref(dw), C.byref(dm))
    return dw.value, dm.value
