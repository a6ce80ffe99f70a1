"""Python binding of libfp.so: frame potentials of random circuit ensembles on MI355X.

Argument marshalling only: every step of the path (sampling, planning of
local random pairs, contraction, reduction, surrogate network) runs in the
library's HIP kernels.  Device buffers are torch tensors on a ROCm device;
PyTorch supplies memory and streams.  The library must be built
(``python paper_2205_09900_amd/build.py``); importing this package without it
raises, and there is no fallback path.
"""

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfp.so")

FP_OK, FP_EINVAL, FP_ETOOBIG, FP_EDEVICE, FP_ENOTIMPL, FP_ENUMERIC = 0, -1, -2, -3, -4, -5
BRICKWORK, LOCAL_RANDOM, HEA, PAULI_CNOT, PAULI_CZ, BRICKWORK_QUDIT = 0, 1, 2, 3, 4, 5
C128, C64, BF16X3 = 0, 1, 2
LAUNCH_AUTO, LAUNCH_WAIT, LAUNCH_WAIT_FREE = 0, 1, 2
CONTINUE, STOP_RESOLVED, STOP_BUDGET = 0, 1, 2

ERROR_NAMES = {FP_EINVAL: "FP_EINVAL", FP_ETOOBIG: "FP_ETOOBIG", FP_EDEVICE: "FP_EDEVICE",
               FP_ENOTIMPL: "FP_ENOTIMPL", FP_ENUMERIC: "FP_ENUMERIC"}

# Symbols declared in include/fp.h.
EXPORTS = [
    "fp_gate_bytes_per_pair", "fp_sample_gates", "fp_workspace_bytes", "fp_contract_trace_batch",
    "fp_frame_potential", "fp_workspace_bytes_groups", "fp_contract_trace_groups",
    "fp_autotune_workspace_bytes", "fp_autotune", "fp_autotune_table", "fp_autotune_load",
    "fp_plan_info", "fp_plan_local_random_host", "fp_plan_program_host", "fp_mlp_param_count", "fp_mlp_act_floats",
    "fp_mlp_init", "fp_mlp_features", "fp_mlp_forward", "fp_mlp_backward", "fp_mlp_adam_step", "fp_mlp_gemm", "fp_mlp_targets", "fp_cv_coefficient", "fp_log_moments",
    "fp_mlp_log_targets", "fp_mlp_link",
    "fp_frame_potential_cv", "fp_frame_potential_noalloc", "fp_cv_holdout", "fp_moments_f32", "fp_cv_choose",
    "fp_cv_time_to_rel_se", "fp_haar_frame_potential", "fp_bootstrap", "fp_layers_to_epsilon",
    "fp_sample_size_decision", "fp_frame_potential_adaptive", "fp_set_launch_mode", "fp_profile_begin", "fp_profile_end", "fp_last_error", "fp_version",
]


class FPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Ensemble(ctypes.Structure):
    _fields_ = [("ansatz", ctypes.c_int32), ("n_qubits", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("local_dim", ctypes.c_int32)]

    def __init__(self, ansatz, n_qubits, depth, local_dim=0):
        super().__init__(int(ansatz), int(n_qubits), int(depth), int(local_dim))

    def __repr__(self):
        q = f", q={self.local_dim}" if self.local_dim else ""
        return f"Ensemble(ansatz={self.ansatz}, n={self.n_qubits}, depth={self.depth}{q})"


class Group(ctypes.Structure):
    _fields_ = [("ensemble_index", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("first_pair", ctypes.c_int64), ("num_pairs", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_2205_09900_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, U64, SZ, D = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_size_t, ctypes.c_double)
    E = ctypes.POINTER(Ensemble)
    sig = {
        "fp_gate_bytes_per_pair": (SZ, [E, I]),
        "fp_sample_gates": (I, [E, I64, U64, U64, I, P, SZ, P]),
        "fp_workspace_bytes": (I, [E, I64, I, ctypes.POINTER(SZ)]),
        "fp_contract_trace_batch": (I, [E, I64, I, P, P, P, SZ, P]),
        "fp_frame_potential": (I, [P, I64, I, P, P, P]),
        "fp_workspace_bytes_groups": (I, [E, I, ctypes.POINTER(Group), I, ctypes.POINTER(SZ)]),
        "fp_contract_trace_groups": (I, [E, I, ctypes.POINTER(Group), I, ctypes.POINTER(P), P, P, SZ, P]),
        "fp_autotune_workspace_bytes": (SZ, [E, I]),
        "fp_autotune": (I, [E, I, P, SZ, ctypes.POINTER(I), P]),
        "fp_autotune_table": (I, [ctypes.c_char_p, SZ]),
        "fp_autotune_load": (I, [ctypes.c_char_p]),
        "fp_plan_info": (I, [E, P, P, P, P]),
        "fp_plan_local_random_host": (I, [I, I, P, P, P, P, P, P]),
        "fp_plan_program_host": (I, [I, I, P, P, P, I64, P, P, P, P]),
        "fp_mlp_param_count": (I64, [I, I]),
        "fp_mlp_act_floats": (I64, [I64, I]),
        "fp_mlp_init": (I, [I, I, U64, P, P]),
        "fp_mlp_features": (I, [E, I64, P, P, P]),
        "fp_mlp_forward": (I, [I, I, I64, P, P, P, P, P]),
        "fp_mlp_backward": (I, [I, I, I64, P, P, P, P, P, P, P]),
        "fp_mlp_adam_step": (I, [I64, P, P, P, I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, P]),
        "fp_mlp_gemm": (I, [I, I, I, P, I, I, P, I, I, P, I, P]),
        "fp_mlp_targets": (I, [P, I64, I, D, P, P]),
        "fp_cv_coefficient": (I, [P, P, I64, I, P, P]),
        "fp_log_moments": (I, [P, I64, D, P, P, P]),
        "fp_mlp_log_targets": (I, [P, I64, D, D, D, P, P]),
        "fp_mlp_link": (I, [P, I64, I, D, D, D, P, P]),
        "fp_frame_potential_cv": (I, [P, P, I64, P, I64, I, D, P, P, P]),
        "fp_set_launch_mode": (I, [I]),
        "fp_haar_frame_potential": (I, [I, D, ctypes.POINTER(D)]),
        "fp_bootstrap": (I, [P, I64, I, I, U64, P, P, P, P, D, P]),
        "fp_layers_to_epsilon": (I, [P, P, I, I, D, D, I, I, I, D, P, ctypes.POINTER(D), ctypes.POINTER(I), P]),
        "fp_sample_size_decision": (I, [D, D, D, D, D, I64, I64, D, D, ctypes.POINTER(I)]),
        "fp_frame_potential_adaptive": (I, [E, I, I, I, U64, I64, I64, D, D, D, D, P, SZ, P, SZ, P, P, P,
                                            ctypes.POINTER(I64), ctypes.POINTER(I), P]),
        "fp_cv_holdout": (I, [P, P, I64, I, P, P]),
        "fp_moments_f32": (I, [P, I64, P, P, P]),
        "fp_cv_choose": (I, [D, D, D, ctypes.POINTER(I), ctypes.POINTER(D)]),
        "fp_cv_time_to_rel_se": (I, [ctypes.POINTER(D), D, D, D, D, D, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "fp_frame_potential_noalloc": (I, [P, I64, I, P, P, P]),
        "fp_profile_begin": (I, []),
        "fp_profile_end": (I, [P, P, P, P]),
        "fp_last_error": (ctypes.c_char_p, []),
        "fp_version": (I, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error():
    return lib.fp_last_error().decode()


def _check(rc):
    if rc != FP_OK:
        raise FPError(rc, last_error())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("expected a device tensor")
        return ctypes.c_void_p(t.data_ptr())
    return t


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ens(e):
    if isinstance(e, Ensemble):
        return e
    return Ensemble(*e)


# ---- C-ABI mirrors (same names, argument marshalling only) --------------------

def fp_gate_bytes_per_pair(ens, precision):
    return int(lib.fp_gate_bytes_per_pair(ctypes.byref(_ens(ens)), int(precision)))


def fp_sample_gates(ens, num_pairs, seed, first_pair, precision, d_gates, stream=None):
    return _check(lib.fp_sample_gates(ctypes.byref(_ens(ens)), int(num_pairs), int(seed), int(first_pair),
                                      int(precision), _ptr(d_gates), d_gates.numel() * d_gates.element_size(),
                                      _stream(stream)))


def fp_workspace_bytes(ens, num_pairs, precision):
    out = ctypes.c_size_t(0)
    _check(lib.fp_workspace_bytes(ctypes.byref(_ens(ens)), int(num_pairs), int(precision), ctypes.byref(out)))
    return int(out.value)


def fp_contract_trace_batch(ens, num_pairs, precision, d_gates, d_trace, d_workspace=None, stream=None):
    wsb = 0 if d_workspace is None else d_workspace.numel() * d_workspace.element_size()
    return _check(lib.fp_contract_trace_batch(ctypes.byref(_ens(ens)), int(num_pairs), int(precision),
                                              _ptr(d_gates), _ptr(d_trace), _ptr(d_workspace), wsb,
                                              _stream(stream)))


def fp_set_launch_mode(mode):
    _check(lib.fp_set_launch_mode(int(mode)))


def fp_frame_potential(d_trace, num_pairs, k_max, stream=None):
    f = (ctypes.c_double * k_max)()
    se = (ctypes.c_double * k_max)()
    _check(lib.fp_frame_potential(_ptr(d_trace), int(num_pairs), int(k_max), f, se, _stream(stream)))
    return list(f), list(se)


def fp_frame_potential_noalloc(d_trace, num_pairs, k_max, stream=None):
    f = (ctypes.c_double * k_max)()
    se = (ctypes.c_double * k_max)()
    _check(lib.fp_frame_potential_noalloc(_ptr(d_trace), int(num_pairs), int(k_max), f, se, _stream(stream)))
    return list(f), list(se)


def fp_frame_potential_cv(d_trace_B, d_g_B, nB, d_g_C, nC, k, c, stream=None):
    f = ctypes.c_double(0)
    se = ctypes.c_double(0)
    _check(lib.fp_frame_potential_cv(_ptr(d_trace_B), _ptr(d_g_B), int(nB), _ptr(d_g_C), int(nC), int(k),
                                     float(c), ctypes.byref(f), ctypes.byref(se), _stream(stream)))
    return f.value, se.value


def fp_plan_info(ens):
    e = _ens(ens)
    bits = (ctypes.c_int32 * max(1, e.n_qubits - 1))()
    peak = ctypes.c_int32(0)
    macs = ctypes.c_double(0)
    ops = ctypes.c_int64(0)
    _check(lib.fp_plan_info(ctypes.byref(e), bits, ctypes.byref(peak), ctypes.byref(macs), ctypes.byref(ops)))
    return {"bits": list(bits), "peak_bits": peak.value, "macs": macs.value, "ops": ops.value}


def fp_plan_local_random_host(n_qubits, bonds_u, bonds_v):
    import numpy as np
    bu = np.ascontiguousarray(bonds_u, dtype=np.int32)
    bv = np.ascontiguousarray(bonds_v, dtype=np.int32)
    if bu.size != bv.size or bu.size < 1:
        raise ValueError("U and V need the same, positive number of steps")
    bits = (ctypes.c_int32 * max(1, n_qubits - 1))()
    peak = ctypes.c_int32(0)
    macs = ctypes.c_double(0)
    ops = ctypes.c_int64(0)
    _check(lib.fp_plan_local_random_host(int(n_qubits), int(bu.size), bu.ctypes.data_as(ctypes.c_void_p),
                                         bv.ctypes.data_as(ctypes.c_void_p), bits, ctypes.byref(peak),
                                         ctypes.byref(macs), ctypes.byref(ops)))
    return {"bits": list(bits), "peak_bits": peak.value, "macs": macs.value, "ops": ops.value}


def fp_mlp_param_count(n_in, hidden):
    return int(lib.fp_mlp_param_count(int(n_in), int(hidden)))


def fp_mlp_act_floats(batch, hidden):
    return int(lib.fp_mlp_act_floats(int(batch), int(hidden)))


def fp_mlp_init(n_in, hidden, seed, d_params, stream=None):
    return _check(lib.fp_mlp_init(int(n_in), int(hidden), int(seed), _ptr(d_params), _stream(stream)))


def fp_mlp_features(ens, num_pairs, d_gates, d_x, stream=None):
    return _check(lib.fp_mlp_features(ctypes.byref(_ens(ens)), int(num_pairs), _ptr(d_gates), _ptr(d_x),
                                      _stream(stream)))


def fp_mlp_forward(n_in, hidden, batch, d_params, d_x, d_y, d_act=None, stream=None):
    return _check(lib.fp_mlp_forward(int(n_in), int(hidden), int(batch), _ptr(d_params), _ptr(d_x), _ptr(d_y),
                                     _ptr(d_act), _stream(stream)))


def fp_mlp_backward(n_in, hidden, batch, d_params, d_x, d_act, d_target, d_grad, want_loss=True, stream=None):
    loss = ctypes.c_double(0)
    _check(lib.fp_mlp_backward(int(n_in), int(hidden), int(batch), _ptr(d_params), _ptr(d_x), _ptr(d_act),
                               _ptr(d_target), _ptr(d_grad), ctypes.byref(loss) if want_loss else None,
                               _stream(stream)))
    return loss.value if want_loss else None


def fp_mlp_adam_step(count, d_params, d_grad, d_adam, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                     stream=None):
    return _check(lib.fp_mlp_adam_step(int(count), _ptr(d_params), _ptr(d_grad), _ptr(d_adam), int(step),
                                       float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def fp_mlp_gemm(M, N, K, d_A, lda, trans_a, d_B, ldb, trans_b, d_C, ldc, stream=None):
    return _check(lib.fp_mlp_gemm(int(M), int(N), int(K), _ptr(d_A), int(lda), int(trans_a), _ptr(d_B), int(ldb),
                                  int(trans_b), _ptr(d_C), int(ldc), _stream(stream)))


def fp_mlp_targets(d_trace, num_pairs, k, scale, d_t, stream=None):
    return _check(lib.fp_mlp_targets(_ptr(d_trace), int(num_pairs), int(k), float(scale), _ptr(d_t),
                                     _stream(stream)))


def fp_cv_coefficient(d_trace, d_g, num_pairs, k, stream=None):
    c = ctypes.c_double(0)
    _check(lib.fp_cv_coefficient(_ptr(d_trace), _ptr(d_g), int(num_pairs), int(k), ctypes.byref(c),
                                 _stream(stream)))
    return c.value


def fp_cv_holdout(d_trace, d_g, num_pairs, k, stream=None):
    """dict with c, rho, mean_f, var_f, mean_g, var_g of a hold-out set."""
    out = (ctypes.c_double * 6)()
    _check(lib.fp_cv_holdout(_ptr(d_trace), _ptr(d_g), int(num_pairs), int(k), out, _stream(stream)))
    return dict(zip(("c", "rho", "mean_f", "var_f", "mean_g", "var_g"), list(out)))


def fp_moments_f32(d_x, n, stream=None):
    m, v = ctypes.c_double(), ctypes.c_double()
    _check(lib.fp_moments_f32(_ptr(d_x), int(n), ctypes.byref(m), ctypes.byref(v), _stream(stream)))
    return m.value, v.value


def fp_cv_choose(rho, sec_per_exact, sec_per_surrogate):
    use, ratio = ctypes.c_int(), ctypes.c_double()
    _check(lib.fp_cv_choose(float(rho), float(sec_per_exact), float(sec_per_surrogate), ctypes.byref(use),
                            ctypes.byref(ratio)))
    return bool(use.value), ratio.value


def fp_cv_time_to_rel_se(stats_B, c, var_g_C, rel_se, sec_per_exact, sec_per_surrogate):
    """stats_B: the dict of fp_cv_holdout on the exact pairs; returns (t_plain, t_cv)."""
    st = (ctypes.c_double * 6)(*[stats_B[k] for k in ("c", "rho", "mean_f", "var_f", "mean_g", "var_g")])
    tp, tc = ctypes.c_double(), ctypes.c_double()
    _check(lib.fp_cv_time_to_rel_se(st, float(c), float(var_g_C), float(rel_se), float(sec_per_exact),
                                    float(sec_per_surrogate), ctypes.byref(tp), ctypes.byref(tc)))
    return tp.value, tc.value


def fp_haar_frame_potential(k, dim):
    out = ctypes.c_double()
    _check(lib.fp_haar_frame_potential(int(k), float(dim), ctypes.byref(out)))
    return out.value


def fp_bootstrap(d_trace, num_pairs, k_max, resamples=300, seed=0, d_samples=None, coverage=0.95, stream=None):
    """Bootstrap of F^(k): (median, lo, hi) lists of k_max values; d_samples (optional device
    tensor of k_max * resamples doubles) receives F^(k) of every resample."""
    med, lo, hi = ((ctypes.c_double * k_max)() for _ in range(3))
    _check(lib.fp_bootstrap(_ptr(d_trace), int(num_pairs), int(k_max), int(resamples), ctypes.c_uint64(seed),
                            _ptr(d_samples), med, lo, hi, float(coverage), _stream(stream)))
    return list(med), list(lo), list(hi)


def fp_layers_to_epsilon(d_F, layers, resamples, F_haar, epsilon, n_qubits, q, k, rel_dev_max=5.0, d_out=None,
                         stream=None):
    """(median layers, failed samples) of the exponential fit over the fit region."""
    lay = (ctypes.c_int32 * len(layers))(*[int(x) for x in layers])
    med, failed = ctypes.c_double(), ctypes.c_int()
    _check(lib.fp_layers_to_epsilon(_ptr(d_F), lay, len(layers), int(resamples), float(F_haar), float(epsilon),
                                    int(n_qubits), int(q), int(k), float(rel_dev_max), _ptr(d_out),
                                    ctypes.byref(med), ctypes.byref(failed), _stream(stream)))
    return med.value, failed.value


def fp_sample_size_decision(F, se, F_haar, F_lower, z, n_done, n_max, seconds, max_seconds):
    d = ctypes.c_int()
    _check(lib.fp_sample_size_decision(float(F), float(se), float(F_haar), float(F_lower), float(z), int(n_done),
                                       int(n_max), float(seconds), float(max_seconds), ctypes.byref(d)))
    return d.value


def fp_frame_potential_adaptive(ens, precision, k_max, k_rule, seed, batch_pairs, max_pairs, max_seconds, z,
                                F_haar, F_lower=-1.0, d_gates=None, d_ws=None, d_trace=None, stream=None):
    """Adaptive estimate: returns (F, SE, pairs used, reason, d_trace)."""
    ens = _ens(ens)
    if d_gates is None:
        d_gates = alloc_gates(ens, batch_pairs, precision)
    if d_ws is None:
        d_ws = workspace(ens, batch_pairs, precision)
    if d_trace is None:
        d_trace = torch.empty(2 * int(max_pairs), dtype=torch.float64, device="cuda")
    f = (ctypes.c_double * k_max)()
    se = (ctypes.c_double * k_max)()
    used, reason = ctypes.c_int64(), ctypes.c_int()
    _check(lib.fp_frame_potential_adaptive(ctypes.byref(ens), int(precision), int(k_max), int(k_rule),
                                           ctypes.c_uint64(seed), int(batch_pairs), int(max_pairs),
                                           float(max_seconds), float(z), float(F_haar), float(F_lower), _ptr(d_gates),
                                           d_gates.numel(), _ptr(d_ws), d_ws.numel(), _ptr(d_trace), f, se,
                                           ctypes.byref(used), ctypes.byref(reason), _stream(stream)))
    return list(f), list(se), used.value, reason.value, d_trace


def fp_log_moments(d_trace, num_pairs, eps=1e-30, stream=None):
    m = ctypes.c_double(0)
    sd = ctypes.c_double(0)
    _check(lib.fp_log_moments(_ptr(d_trace), int(num_pairs), float(eps), ctypes.byref(m), ctypes.byref(sd),
                              _stream(stream)))
    return m.value, sd.value


def fp_mlp_log_targets(d_trace, num_pairs, eps, mean, std_dev, d_t, stream=None):
    return _check(lib.fp_mlp_log_targets(_ptr(d_trace), int(num_pairs), float(eps), float(mean), float(std_dev),
                                         _ptr(d_t), _stream(stream)))


def fp_mlp_link(d_y, n, k, mean, std_dev, shift, d_g, stream=None):
    return _check(lib.fp_mlp_link(_ptr(d_y), int(n), int(k), float(mean), float(std_dev), float(shift), _ptr(d_g),
                                  _stream(stream)))


def _groups_args(ensembles, groups):
    E = (Ensemble * len(ensembles))(*[_ens(e) for e in ensembles])
    G = (Group * len(groups))()
    for i, g in enumerate(groups):
        G[i].ensemble_index, G[i].precision, G[i].first_pair, G[i].num_pairs = (int(x) for x in g)
    return E, G


def fp_workspace_bytes_groups(ensembles, groups):
    """ensembles: list of (ansatz, n, depth); groups: list of (ensemble_index, precision, first_pair, num_pairs)."""
    E, G = _groups_args(ensembles, groups)
    out = ctypes.c_size_t(0)
    _check(lib.fp_workspace_bytes_groups(E, len(ensembles), G, len(groups), ctypes.byref(out)))
    return int(out.value)


def fp_contract_trace_groups(ensembles, groups, gate_buffers, d_trace, d_ws, stream=None):
    E, G = _groups_args(ensembles, groups)
    ptrs = (ctypes.c_void_p * len(groups))(*[g.data_ptr() for g in gate_buffers])
    wsb = d_ws.numel() * d_ws.element_size()
    return _check(lib.fp_contract_trace_groups(E, len(ensembles), G, len(groups), ptrs, _ptr(d_trace), _ptr(d_ws),
                                               wsb, _stream(stream)))


def fp_autotune_workspace_bytes(ens, precision):
    return int(lib.fp_autotune_workspace_bytes(ctypes.byref(_ens(ens)), int(precision)))


def fp_autotune(ens, precision, d_ws=None, stream=None):
    if d_ws is None:
        d_ws = torch.empty(max(256, fp_autotune_workspace_bytes(ens, precision)), dtype=torch.uint8, device="cuda")
    choice = ctypes.c_int(-1)
    _check(lib.fp_autotune(ctypes.byref(_ens(ens)), int(precision), _ptr(d_ws),
                           d_ws.numel() * d_ws.element_size(), ctypes.byref(choice), _stream(stream)))
    return choice.value


# fp_autotune's choices: 3 * lane class + task size
AUTOTUNE_CLASSES = ("tiny", "small", "mid", "large")
AUTOTUNE_TASK_FLOPS = (5e6, 2e7, 8e7)


def fp_autotune_table():
    buf = ctypes.create_string_buffer(1 << 20)
    _check(lib.fp_autotune_table(buf, len(buf)))
    return buf.value.decode()


def fp_autotune_load(text):
    return _check(lib.fp_autotune_load(text.encode()))


# Launch classes of fp_profile_end (include/fp.h).  For local random batches
# classes 0 and 1 are the one-wavefront-per-pair sweeps (registers up to 2^8
# and 2^10 entries); for fixed topologies they are 16- and 64-lane tiles.
KERNEL_CLASSES = ("lds16", "lds64", "lds256", "lds1024", "hbm", "hea", "plan", "prep", "sample")


def fp_profile_begin():
    return _check(lib.fp_profile_begin())


def fp_profile_end():
    k = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * k)()
    n = (ctypes.c_int64 * k)()
    fl = (ctypes.c_double * k)()
    by = (ctypes.c_double * k)()
    _check(lib.fp_profile_end(ms, n, fl, by))
    return {c: {"ms": ms[i], "launches": n[i], "flops": fl[i], "bytes": by[i]} for i, c in enumerate(KERNEL_CLASSES)}


OP_DTYPE = [("type", "u1"), ("p", "u1"), ("q", "u1"), ("bits", "u1"), ("arg", "<i4")]


def fp_plan_program_host(n_qubits, bonds_u, bonds_v):
    import numpy as np
    bu = np.ascontiguousarray(bonds_u, dtype=np.int32)
    bv = np.ascontiguousarray(bonds_v, dtype=np.int32)
    if bu.size != bv.size or bu.size < 1:
        raise ValueError("U and V need the same, positive number of steps")
    s = int(bu.size)
    max_ops = 10 * s + n_qubits + 8
    ops = np.zeros(max_ops, dtype=OP_DTYPE)
    wg = np.zeros((2 * s, 2), dtype=np.int32)
    fac = np.zeros(2 * s, dtype=np.int32)
    nops = ctypes.c_int64(0)
    l2 = ctypes.c_int32(0)
    v = ctypes.c_void_p
    _check(lib.fp_plan_program_host(int(n_qubits), s, bu.ctypes.data_as(v), bv.ctypes.data_as(v),
                                    ops.ctypes.data_as(v), max_ops, wg.ctypes.data_as(v), fac.ctypes.data_as(v),
                                    ctypes.byref(nops), ctypes.byref(l2)))
    return ops[: nops.value], wg, fac, l2.value


# ---- convenience -------------------------------------------------------------------

def alloc_gates(ens, num_pairs, precision, device="cuda"):
    nb = fp_gate_bytes_per_pair(ens, precision)
    if nb == 0:
        raise FPError(FP_EINVAL, "invalid ensemble or precision")
    return torch.empty(int(num_pairs) * nb, dtype=torch.uint8, device=device)


def sample(ens, num_pairs, seed, first_pair=0, precision=C64, device="cuda", stream=None):
    g = alloc_gates(ens, num_pairs, precision, device)
    fp_sample_gates(ens, num_pairs, seed, first_pair, precision, g, stream)
    return g


def workspace(ens, num_pairs, precision, device="cuda"):
    nb = fp_workspace_bytes(ens, num_pairs, precision)
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)


def contract(ens, gates, num_pairs, precision, ws=None, stream=None):
    """Traces of num_pairs pairs as a complex128 tensor."""
    tr = torch.empty(2 * int(num_pairs), dtype=torch.float64, device=gates.device)
    if ws is None:
        ws = workspace(ens, num_pairs, precision, gates.device)
    fp_contract_trace_batch(ens, num_pairs, precision, gates, tr, ws, stream)
    return torch.view_as_complex(tr.view(-1, 2))


def frame_potential(traces, k_max, stream=None):
    t = torch.view_as_real(traces).reshape(-1) if traces.is_complex() else traces
    return fp_frame_potential(t, t.numel() // 2, k_max, stream)
