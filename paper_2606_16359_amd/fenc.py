"""Python binding of the C ABI in include/fenc.h (argument marshalling only).

PyTorch provides device memory and the current HIP stream; every step of the
homomorphic computation runs in the library's kernels.  Loading fails loudly
when the HIP library has not been built.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

FENC_LAYOUT_FRAGMENT, FENC_LAYOUT_VECTOR = 0, 1
FENC_MODE_BATCHED, FENC_MODE_PER_OP = 0, 1
FENC_ENOMEM = -2
RELIN = -(1 << 31)

STATUS = {0: "FENC_OK", -1: "FENC_EINVAL", -2: "FENC_ENOMEM", -3: "FENC_ENOKEY", -4: "FENC_ELEVEL",
          -5: "FENC_ESCALE", -6: "FENC_ELAYOUT", -7: "FENC_EHIP", -8: "FENC_EUNSUPPORTED"}


class FencError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("q_bits", C.c_uint32), ("n_p", C.c_uint32),
                ("p_bits", C.c_uint32), ("dnum", C.c_uint32), ("log2_scale", C.c_double), ("seed", C.c_uint64)]


class Layout(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("kind", "bs", "c", "h", "w", "M", "S", "m", "bs_g", "chan_per_ct",
                                         "n_bg", "n_cg", "replicate", "dil", "level", "d", "n_feat")] + \
               [("scale", C.c_double), ("map_id", C.c_uint64)]

    def n_ct(self):
        if self.kind == 2:   # token fragments
            return self.n_bg * self.S * self.n_cg
        return self.n_bg * self.n_cg * self.S * self.S if self.kind == 0 else self.n_bg

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}

    def copy(self):
        out = Layout()
        C.pointer(out)[0] = self
        return out


class CtBatch(C.Structure):
    _fields_ = [("data", C.c_void_p), ("lay", Layout)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("rot_inner", "rot_outer", "rot_other", "keyswitch", "modup", "moddown",
                                         "ntt_limbs", "intt_limbs", "pmult", "smult", "rescale", "relin",
                                         "launches", "cts_out")]


_LIBS = {}


def load(path=None):
    """Load the library (default: the in-tree HIP build)."""
    hip = path is None
    path = path or _build.LIB
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise RuntimeError(f"FEnc HIP library not built: {path} (run __graft_entry__.build())")
    if hip:
        # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
        # first makes the dynamic loader bind this library to the same runtime,
        # so there is one HIP runtime per process and library launches on torch
        # streams can be captured into torch's hipGraphs.
        import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, u32, d, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_double, C.c_uint64
    P, L, B = C.POINTER(Params), C.POINTER(Layout), C.POINTER(CtBatch)
    sig = {
        "fenc_last_error": (C.c_char_p, []),
        "fenc_ctx_create": (C.c_int, [P, C.POINTER(vp)]),
        "fenc_ctx_create_server": (C.c_int, [P, C.POINTER(vp)]),
        "fenc_ctx_destroy": (None, [vp]),
        "fenc_ctx_primes": (C.c_int, [vp, vp]),
        "fenc_set_mode": (C.c_int, [vp, C.c_int]),
        "fenc_set_plaintext_budget": (C.c_int, [vp, C.c_int64]),
        "fenc_set_own_copy_limit": (C.c_int, [vp, C.c_int64]),
        "fenc_set_workspace_limit": (C.c_int, [vp, C.c_int64]),
        "fenc_stats": (C.c_int, [vp, C.POINTER(Counters)]),
        "fenc_profile_kernel": (C.c_int, [vp, C.c_char_p]),
        "fenc_profile_result": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "fenc_profile_summary": (C.c_int, [vp, C.c_char_p, C.c_int64]),
        "fenc_stats_reset": (None, [vp]),
        "fenc_device_bytes": (C.c_int64, [vp]),
        "fenc_keygen": (C.c_int, [vp, vp, u32, C.c_int, C.c_int]),
        "fenc_key_export": (C.c_int, [vp, i32, vp]),
        "fenc_key_list": (C.c_int, [vp, vp, C.c_int32]),
        "fenc_key_export_galois": (C.c_int, [vp, C.c_uint64, vp]),
        "fenc_key_import": (C.c_int, [vp, C.c_uint64, vp]),
        "fenc_plan_layout": (C.c_int, [vp, u32, u32, u32, u32, u32, u32, i32, L]),
        "fenc_plan_network": (C.c_int, [vp, u32, u32, u32, u32, vp, u32, i32, vp, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int64)]),
        "fenc_conv2d_keyswitches": (C.c_int, [vp, L, u32, u32, u32, u32, u32, C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "fenc_compress_keyswitches": (C.c_int, [vp, L, vp, C.POINTER(C.c_int64)]),
        "fenc_plan_tokens": (C.c_int, [vp, u32, u32, u32, u32, L]),
        "fenc_layout_n_ct": (C.c_int, [L]),
        "fenc_ct_bytes": (C.c_int64, [vp, L]),
        "fenc_layout_slot": (C.c_int, [vp, L, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(i32), C.POINTER(i32)]),
        "fenc_layout_map": (C.c_int, [vp, L, vp]),
        "fenc_encode_fragment": (C.c_int, [vp, vp, L, vp]),
        "fenc_encode_slots": (C.c_int, [vp, vp, i32, d, vp]),
        "fenc_encrypt": (C.c_int, [vp, vp, L, u64, B, vp]),
        "fenc_decrypt": (C.c_int, [vp, B, vp, vp]),
        "fenc_decrypt_raw": (C.c_int, [vp, B, vp, vp]),
        "fenc_ct_export": (C.c_int, [vp, B, vp, vp]),
        "fenc_ct_import": (C.c_int, [vp, vp, B, vp]),
        "fenc_conv2d": (C.c_int, [vp, B, vp, vp, u32, u32, u32, u32, u32, C.c_int32, B, vp]),
        "fenc_avgpool2": (C.c_int, [vp, B, B, vp]),
        "fenc_poly_act": (C.c_int, [vp, B, vp, u32, B, vp]),
        "fenc_compress": (C.c_int, [vp, B, L, B, vp]),
        "fenc_fc": (C.c_int, [vp, B, vp, vp, u32, B, vp]),
        "fenc_rotate": (C.c_int, [vp, B, vp, u32, B, vp]),
        "fenc_rotate_sum": (C.c_int, [vp, B, B, vp, u32, B, vp]),
        "fenc_rescale": (C.c_int, [vp, B, B, vp]),
        "fenc_rescale_noalloc": (C.c_int, [vp, B, B, vp]),
        "fenc_ntt_rows": (C.c_int, [vp, vp, vp, u32, C.c_int]),
        "fenc_ntt_config": (C.c_int, [vp, vp]),
        "fenc_set_hoisting": (C.c_int, [vp, C.c_int]),
        "fenc_last_hoisting": (C.c_int, [vp]),
        "fenc_set_baby_step": (C.c_int, [vp, C.c_int]),
        "fenc_last_baby_step": (C.c_int, [vp]),
        "fenc_set_ntt_config": (C.c_int, [vp, vp]),
        "fenc_sample_word": (u64, [u64, u64, u64]),
        "fenc_sample_gauss": (C.c_int, [u64, u64, u64]),
        "fenc_encode_int": (C.c_int, [i32, vp, d, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    _LIBS[path] = lib
    return lib


def _ptr(a):
    return a.ctypes.data if isinstance(a, np.ndarray) else a.data_ptr()


class Ciphertexts:
    """A ciphertext batch: device buffer + layout."""

    def __init__(self, fenc, lay, buf):
        self.fenc, self.lay, self.buf = fenc, lay, buf

    def struct(self):
        b = CtBatch()
        b.data = _ptr(self.buf) if self.buf is not None else None
        b.lay = self.lay
        return b

    @property
    def n_ct(self):
        return self.lay.n_ct()

    def shape(self):
        return (self.n_ct, 2, self.lay.level + 1, self.fenc.N)


class Fenc:
    """One library context.  `lib_path` selects another build of the same ABI
    (the CPU test suite uses the kernel emulator); the default is the HIP library."""

    def __init__(self, log_n, n_q, q_bits, n_p, p_bits, dnum, log2_scale, seed, lib_path=None, server=False):
        """server=True: a context without a secret key (evaluation keys are
        imported with key_import)."""
        self.lib = load(lib_path)
        self.emulated = lib_path is not None and "emu" in os.path.basename(lib_path)
        p = Params(log_n, n_q, q_bits, n_p, p_bits, dnum, log2_scale, seed)
        h = C.c_void_p()
        create = self.lib.fenc_ctx_create_server if server else self.lib.fenc_ctx_create
        self._check(create(C.byref(p), C.byref(h)))
        self.h = h
        self.params = p
        self.N, self.ns, self.L = 1 << log_n, 1 << (log_n - 1), n_q - 1
        self.n_q, self.n_p, self.dnum = n_q, n_p, dnum
        self.alpha = (n_q + dnum - 1) // dnum
        self.hoist = 1

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.fenc_ctx_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise FencError(rc, self.lib.fenc_last_error().decode())

    # ------------------------------------------------------------ memory
    def _stream(self):
        if self.emulated:
            return None
        import torch
        return torch.cuda.current_stream().cuda_stream

    def alloc(self, n_u64):
        if self.emulated:
            return np.zeros(max(1, n_u64), np.uint64)
        import torch
        return torch.empty(max(1, n_u64), dtype=torch.int64, device="cuda")

    def alloc_cts(self, lay):
        n = lay.n_ct() * 2 * (lay.level + 1) * self.N
        return Ciphertexts(self, lay, self.alloc(n))

    # ------------------------------------------------------------ context
    def primes(self):
        out = np.zeros(self.n_q + self.n_p, np.uint64)
        self._check(self.lib.fenc_ctx_primes(self.h, out.ctypes.data))
        return [int(x) for x in out]

    def set_mode(self, mode):
        self._check(self.lib.fenc_set_mode(self.h, mode))

    def set_hoisting(self, mode):
        """1: linear combinations of rotated copies in the extended basis (one
        ModDown per combined ciphertext); 0: one ModDown per rotated copy;
        2: per layer, the schedule with the smaller modelled HBM traffic
        (last_hoisting() tells which one a layer ran with)."""
        self._check(self.lib.fenc_set_hoisting(self.h, mode))
        self.hoist = mode

    def set_baby_step(self, n1):
        """Baby step of convolutions' outer rotations: 1 (default) the plain
        form, n1 > 1 fixed, 0 chosen per layer by key-switch count."""
        self._check(self.lib.fenc_set_baby_step(self.h, n1))

    def last_baby_step(self):
        """Baby step the most recent conv2d ran with."""
        return self.lib.fenc_last_baby_step(self.h)

    def last_hoisting(self):
        """Schedule (0/1) of the most recent conv2d / avgpool2 / compress."""
        return self.lib.fenc_last_hoisting(self.h)

    def ntt_config(self):
        out = np.zeros(8, np.int32)
        self._check(self.lib.fenc_ntt_config(self.h, out.ctypes.data))
        return [tuple(int(v) for v in out[2 * k:2 * k + 2]) for k in range(4)]

    def set_ntt_config(self, cfg):
        arr = np.array([v for pair in cfg for v in pair], np.int32)
        self._check(self.lib.fenc_set_ntt_config(self.h, arr.ctypes.data))

    def set_plaintext_budget(self, nbytes):
        self._check(self.lib.fenc_set_plaintext_budget(self.h, nbytes))

    def set_own_copy_limit(self, nbytes):
        self._check(self.lib.fenc_set_own_copy_limit(self.h, nbytes))

    def set_workspace_limit(self, nbytes):
        self._check(self.lib.fenc_set_workspace_limit(self.h, nbytes))

    def stats(self):
        c = Counters()
        self._check(self.lib.fenc_stats(self.h, C.byref(c)))
        return {n: getattr(c, n) for n, _ in c._fields_}

    def profile_kernel(self, name):
        self._check(self.lib.fenc_profile_kernel(self.h, name.encode() if name else None))

    def profile_summary(self):
        """Per-kernel {name: (total_ms, launches, bytes, modmuls)} after profile_kernel("*")."""
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.fenc_profile_summary(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, ms, n, b, o = line.split()
            out[name] = (float(ms), int(n), float(b), float(o))
        return out

    def profile_result(self):
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        self._check(self.lib.fenc_profile_result(self.h, C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def stats_reset(self):
        self.lib.fenc_stats_reset(self.h)

    def device_bytes(self):
        return self.lib.fenc_device_bytes(self.h)

    def keygen(self, rot_steps=(), relin=True, strict=False):
        arr = np.array(list(rot_steps), np.int32)
        self._check(self.lib.fenc_keygen(self.h, arr.ctypes.data if len(arr) else None, len(arr), int(relin),
                                         int(strict)))

    def key_list(self):
        n = self.lib.fenc_key_list(self.h, None, 0)
        if n < 0:
            self._check(n)
        out = np.zeros(max(1, n), np.uint64)
        self.lib.fenc_key_list(self.h, out.ctypes.data, n)
        return [int(g) for g in out[:n]]

    def _key_shape(self):
        ndig = (self.n_q + self.alpha - 1) // self.alpha
        return (ndig, 2, self.n_q + self.n_p, self.N)

    def key_export_galois(self, g):
        out = np.zeros(self._key_shape(), np.uint64)
        self._check(self.lib.fenc_key_export_galois(self.h, g, out.ctypes.data))
        return out

    def key_import(self, g, key):
        key = np.ascontiguousarray(key, np.uint64)
        assert key.shape == self._key_shape()
        self._check(self.lib.fenc_key_import(self.h, g, key.ctypes.data))

    def key_export(self, shift):
        ndig = (self.n_q + self.alpha - 1) // self.alpha
        out = np.zeros((ndig, 2, self.n_q + self.n_p, self.N), np.uint64)
        self._check(self.lib.fenc_key_export(self.h, shift, out.ctypes.data))
        return out

    # ------------------------------------------------------------ layouts
    def plan_layout(self, bs, c, h, w, k_next, cout_next, s_override=0):
        lay = Layout()
        self._check(self.lib.fenc_plan_layout(self.h, bs, c, h, w, k_next, cout_next, s_override, C.byref(lay)))
        return lay

    LAYER_KINDS = {"conv": 0, "pool": 1, "act": 2, "compress": 3}

    def plan_network(self, bs, shape, layers, max_repacks=1):
        """Block size per layer of a chain (dicts with kind "conv" (cout, k,
        stride=1, pad=0, groups=1), "pool", "act" (k: degree, default 2) or
        "compress"); returns (block sizes, key switches, MAC terms)."""
        arr = np.zeros((len(layers), 6), np.int32)
        for i, ly in enumerate(layers):
            arr[i] = [self.LAYER_KINDS[ly["kind"]], ly.get("cout", 0), ly.get("k", 0), ly.get("stride", 1),
                      ly.get("pad", 0), ly.get("groups", 1)]
        out = np.zeros(len(layers), np.int32)
        ks, tm = C.c_int64(), C.c_int64()
        c, h, w = shape
        self._check(self.lib.fenc_plan_network(self.h, bs, c, h, w, arr.ctypes.data, len(layers), max_repacks,
                                               out.ctypes.data, C.byref(ks), C.byref(tm)))
        return [int(v) for v in out], ks.value, tm.value

    def conv2d_keyswitches(self, lay, cout, k, stride=1, pad=0, groups=1):
        """(inner, outer) key switches and scalar MAC terms conv2d performs on
        layout lay."""
        a, b, t = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.fenc_conv2d_keyswitches(self.h, C.byref(lay), cout, k, stride, pad, groups, C.byref(a),
                                                     C.byref(b), C.byref(t)))
        return a.value, b.value, t.value

    def conv2d_layout(self, lay, cout, k, stride=1, pad=0, groups=1):
        """Output layout of conv2d on layout lay (the sizing call; nothing is
        built or run)."""
        b, out = CtBatch(), CtBatch()
        b.data, b.lay, out.data = None, lay, None
        w = np.zeros(cout * (lay.c // groups) * k * k)
        self._check(self.lib.fenc_conv2d(self.h, C.byref(b), w.ctypes.data, None, cout, k, stride, pad, groups, 0,
                                         C.byref(out), None))
        return out.lay.copy()

    def avgpool2_layout(self, lay):
        b, out = CtBatch(), CtBatch()
        b.data, b.lay, out.data = None, lay, None
        self._check(self.lib.fenc_avgpool2(self.h, C.byref(b), C.byref(out), None))
        return out.lay.copy()

    def compress_keyswitches(self, lay, target=None):
        ks = C.c_int64()
        self._check(self.lib.fenc_compress_keyswitches(self.h, C.byref(lay), C.byref(target) if target else None,
                                                       C.byref(ks)))
        return ks.value

    def plan_tokens(self, n, E, S, group=0):
        """Token-fragment layout: n tokens of E features in S fragments."""
        lay = Layout()
        self._check(self.lib.fenc_plan_tokens(self.h, n, E, S, group, C.byref(lay)))
        return lay

    def layout_slot(self, lay, b, ch, y, x):
        ct, slot = C.c_int32(), C.c_int32()
        self._check(self.lib.fenc_layout_slot(self.h, C.byref(lay), b, ch, y, x, C.byref(ct), C.byref(slot)))
        return ct.value, slot.value

    def layout_map(self, lay):
        out = np.zeros(max(1, lay.n_feat), np.int32)
        self._check(self.lib.fenc_layout_map(self.h, C.byref(lay), out.ctypes.data))
        return out[:lay.n_feat]

    # ------------------------------------------------------------ client side
    def encode_fragment(self, x, lay):
        x = np.ascontiguousarray(x, np.float64)
        out = np.zeros((lay.n_ct(), lay.level + 1, self.N), np.uint64)
        self._check(self.lib.fenc_encode_fragment(self.h, x.ctypes.data, C.byref(lay), out.ctypes.data))
        return out

    def encode_slots(self, z, level, scale):
        z = np.ascontiguousarray(z, np.float64)
        out = np.zeros((level + 1, self.N), np.uint64)
        self._check(self.lib.fenc_encode_slots(self.h, z.ctypes.data, level, scale, out.ctypes.data))
        return out

    def encrypt(self, pt, lay, seed):
        pt = np.ascontiguousarray(pt, np.uint64)
        ct = self.alloc_cts(lay)
        b = ct.struct()
        self._check(self.lib.fenc_encrypt(self.h, pt.ctypes.data, C.byref(lay), seed, C.byref(b), self._stream()))
        return ct

    def decrypt(self, ct):
        L = ct.lay
        x = np.zeros((L.bs, L.c, L.h, L.w))
        b = ct.struct()
        self._check(self.lib.fenc_decrypt(self.h, C.byref(b), x.ctypes.data, self._stream()))
        return x

    def decrypt_raw(self, ct):
        out = np.zeros((ct.n_ct, ct.lay.level + 1, self.N), np.uint64)
        b = ct.struct()
        self._check(self.lib.fenc_decrypt_raw(self.h, C.byref(b), out.ctypes.data, self._stream()))
        return out

    def export(self, ct):
        out = np.zeros(ct.shape(), np.uint64)
        b = ct.struct()
        self._check(self.lib.fenc_ct_export(self.h, C.byref(b), out.ctypes.data, self._stream()))
        return out

    def import_cts(self, host, lay):
        host = np.ascontiguousarray(host, np.uint64)
        ct = self.alloc_cts(lay)
        b = ct.struct()
        self._check(self.lib.fenc_ct_import(self.h, host.ctypes.data, C.byref(b), self._stream()))
        return ct

    # ------------------------------------------------------------ server side
    def _op(self, fn, *args, keep=None):
        """Two-call convention: size the output, allocate it, run.  When the
        library's workspace allocation fails, the cached blocks PyTorch holds
        are returned to the device and the call is made once more (an
        operation reads only its input and writes only its output, so running
        it again is safe)."""
        out = CtBatch()
        out.data = None
        self._check(fn(*args, C.byref(out), self._stream()))
        res = self.alloc_cts(out.lay.copy())
        ob = res.struct()
        rc = fn(*args, C.byref(ob), self._stream())
        if rc == FENC_ENOMEM and not self.emulated:
            import torch
            if torch.cuda.is_current_stream_capturing():
                self._check(rc)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            rc = fn(*args, C.byref(ob), self._stream())
        self._check(rc)
        return res

    def conv2d(self, ct, w, stride=1, pad=0, groups=1, bias=None, s_out=0):
        """s_out > 0: the output goes straight into the fragment layout of block
        size s_out (the compression repack fused with the convolution)."""
        w = np.ascontiguousarray(w, np.float64)
        bv = None if bias is None else np.ascontiguousarray(bias, np.float64)
        b = ct.struct()
        return self._op(self.lib.fenc_conv2d, self.h, C.byref(b), w.ctypes.data,
                        None if bv is None else bv.ctypes.data, w.shape[0], w.shape[2], stride, pad, groups, s_out,
                        keep=bv)

    def avgpool2(self, ct):
        b = ct.struct()
        return self._op(self.lib.fenc_avgpool2, self.h, C.byref(b))

    def poly_act(self, ct, coeffs=(0.0, 0.0, 1.0), inplace=False):
        """inplace: the output overwrites the input's buffer (the input batch
        must not be used afterwards)."""
        c = np.ascontiguousarray(coeffs, np.float64)
        b = ct.struct()
        if not inplace:
            return self._op(self.lib.fenc_poly_act, self.h, C.byref(b), c.ctypes.data, len(c) - 1)
        out = CtBatch()
        out.data = None
        self._check(self.lib.fenc_poly_act(self.h, C.byref(b), c.ctypes.data, len(c) - 1, C.byref(out),
                                           self._stream()))
        res = Ciphertexts(self, out.lay.copy(), ct.buf)
        ob = res.struct()
        self._check(self.lib.fenc_poly_act(self.h, C.byref(b), c.ctypes.data, len(c) - 1, C.byref(ob),
                                           self._stream()))
        return res

    def compress(self, ct, target=None):
        """target: a Layout of the same tensor (None: the library's vector)."""
        b = ct.struct()
        t = None if target is None else target.copy()
        return self._op(self.lib.fenc_compress, self.h, C.byref(b), None if t is None else C.byref(t))

    def fc(self, ct, w, bias=None):
        w = np.ascontiguousarray(w, np.float64)
        bv = None if bias is None else np.ascontiguousarray(bias, np.float64)
        b = ct.struct()
        return self._op(self.lib.fenc_fc, self.h, C.byref(b), w.ctypes.data, None if bv is None else bv.ctypes.data,
                        w.shape[0], keep=bv)

    def rescale(self, ct):
        b = ct.struct()
        return self._op(self.lib.fenc_rescale, self.h, C.byref(b))

    def rescale_noalloc(self, ct, out=None):
        """The rescale through the library's static scratch (no device
        allocation by the library); out: a preallocated output batch."""
        b = ct.struct()
        if out is None:
            o = CtBatch()
            o.data = None
            self._check(self.lib.fenc_rescale_noalloc(self.h, C.byref(b), C.byref(o), self._stream()))
            out = self.alloc_cts(o.lay.copy())
        ob = out.struct()
        self._check(self.lib.fenc_rescale_noalloc(self.h, C.byref(b), C.byref(ob), self._stream()))
        return out

    def rotate(self, ct, shifts):
        sh = np.array(shifts, np.int32)
        lay = ct.lay.copy()
        lay.n_bg *= len(sh)      # container layout: n_ct * len(shifts) ciphertexts, ct-major
        out = Ciphertexts(self, lay, self.alloc(ct.n_ct * len(sh) * 2 * (lay.level + 1) * self.N))
        ib, ob = ct.struct(), out.struct()
        self._check(self.lib.fenc_rotate(self.h, C.byref(ib), sh.ctypes.data, len(sh), C.byref(ob), self._stream()))
        return out

    def rotate_sum(self, z0, zs, shifts):
        sh = np.array(shifts, np.int32)
        lay = zs.lay.copy()
        lay.n_bg, lay.n_cg, lay.S = 1, 1, 1      # container layout: one ciphertext
        out = Ciphertexts(self, lay, self.alloc(2 * (lay.level + 1) * self.N))
        zb, ob = zs.struct(), out.struct()
        z0b = z0.struct() if z0 is not None else None
        self._check(self.lib.fenc_rotate_sum(self.h, C.byref(z0b) if z0b is not None else None, C.byref(zb),
                                             sh.ctypes.data, len(sh), C.byref(ob), self._stream()))
        return out

    def ntt_rows(self, rows, primes, inverse=False):
        rows = np.array(rows, np.uint64)
        pr = np.array(primes, np.int32)
        self._check(self.lib.fenc_ntt_rows(self.h, rows.ctypes.data, pr.ctypes.data, len(pr), int(inverse)))
        return rows

    def synchronize(self):
        if not self.emulated:
            import torch
            torch.cuda.synchronize()


def sample_word(seed, tag, i, lib_path=None):
    return load(lib_path).fenc_sample_word(seed, tag, i)


def sample_gauss(seed, tag, i, lib_path=None):
    return load(lib_path).fenc_sample_gauss(seed, tag, i)


def encode_int(log_n, z, scale, lib_path=None):
    z = np.ascontiguousarray(z, np.float64)
    out = np.zeros(1 << log_n, np.int64)
    rc = load(lib_path).fenc_encode_int(log_n, z.ctypes.data, scale, out.ctypes.data)
    if rc:
        raise FencError(rc, load(lib_path).fenc_last_error().decode())
    return out
