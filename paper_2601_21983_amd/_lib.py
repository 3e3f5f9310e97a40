"""ctypes binding of libsmc.so (argument marshalling only).

Every function here has the name and argument order of the C entry point in
include/smc.h.  Device pointers are plain integers (``tensor.data_ptr()``);
streams are ``hipStream_t`` integers (``torch.cuda.current_stream().cuda_stream``).
Each call raises ``SMCError`` on a non-OK status.  The library must be built
(``python paper_2601_21983_amd/build.py``); importing this module without it
raises ``ImportError`` - there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsmc.so")

SMC_MAX_LAYERS = 8
SMC_ACT_TANH, SMC_ACT_RELU = 0, 1
SMC_LIK_CATEGORICAL, SMC_LIK_GAUSSIAN = 0, 1
SMC_PREC_FP32, SMC_PREC_BF16, SMC_PREC_BF16X3 = 0, 1, 2
SMC_PROPOSAL_FIXED, SMC_PROPOSAL_LEARNED = 0, 1
SMC_MODEL_MLP, SMC_MODEL_CNN, SMC_MODEL_LENET = 0, 1, 2
SMC_RESAMPLE_IF_NEEDED, SMC_RESAMPLE_ALWAYS, SMC_RESAMPLE_NEVER = 0, 1, 2

STATUS = {0: "SMC_OK", 1: "SMC_ERR_ARG", 2: "SMC_ERR_OOM", 3: "SMC_ERR_DEVICE", 4: "SMC_ERR_STATE",
          5: "SMC_ERR_NONFINITE", 6: "SMC_ERR_UNSUPPORTED", 7: "SMC_ERR_NOLIB"}


class smc_config(C.Structure):
    _fields_ = [
        ("n_particles", C.c_int32),
        ("n_layers", C.c_int32),
        ("widths", C.c_int32 * (SMC_MAX_LAYERS + 1)),
        ("activation", C.c_int32),
        ("model_kind", C.c_int32),
        ("likelihood", C.c_int32),
        ("precision", C.c_int32),
        ("proposal", C.c_int32),
        ("leapfrog_steps", C.c_int32),
        ("n_iterations", C.c_int32),
        ("step_size", C.c_double),
        ("prior_std", C.c_double),
        ("noise_std", C.c_double),
        ("ess_frac", C.c_double),
        ("seed", C.c_uint64),
        ("act_budget_bytes", C.c_int64),
    ]


class smc_step_info(C.Structure):
    _fields_ = [
        ("ess", C.c_double),
        ("log_z_increment", C.c_double),
        ("mean_loglik", C.c_double),
        ("max_loglik", C.c_double),
        ("n_nonfinite", C.c_int32),
        ("resample_recommended", C.c_int32),
        ("grad_evals", C.c_int64),
    ]


class SMCError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2601_21983_amd/build.py`")
# PyTorch ships its own HIP runtime (soname libamdhip64.so.7) and its libraries ask for it as
# libamdhip64.so.  Loading torch first makes libsmc.so's libamdhip64.so.7 resolve to that same
# runtime; loading libsmc.so first would bring in the system runtime and torch would then load
# a second one, whose device memory and streams this library could not use.
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI itself does not need torch
    pass

lib = C.CDLL(LIB_PATH)

_vp, _i32, _i64, _u32, _u64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
_handle = C.c_void_p

_SIGS = {
    "smc_status_string": (C.c_char_p, [_i32]),
    "smc_last_error": (C.c_char_p, []),
    "smc_init": (_i32, [C.POINTER(smc_config), _vp, _vp, _i64, _vp, _i64, _d, _vp, C.POINTER(_handle)]),
    "smc_destroy": (None, [_handle]),
    "smc_step": (_i32, [_handle, _i64, _d, C.POINTER(smc_step_info)]),
    "smc_step_tempered": (_i32, [_handle, _i64, _i64, _d, _d, C.POINTER(smc_step_info)]),
    "smc_segment_moments": (_i32, [_handle, C.POINTER(_d)]),
    "smc_resample": (_i32, [_handle, _i32, C.POINTER(_d), C.POINTER(_i32), C.POINTER(_i32)]),
    "smc_resample_multinomial": (_i32, [_handle, _i32, _vp, C.POINTER(_i32), C.POINTER(_i32)]),
    "smc_posterior_predict": (_i32, [_handle, _vp, _vp, _i64, _vp, C.POINTER(_d), C.POINTER(_d)]),
    "smc_posterior_mean": (_i32, [_handle, _vp]),
    "smc_posterior_mean_change": (_i32, [_handle, C.POINTER(_d)]),
    "smc_get_state": (_i32, [_handle, _vp, _vp, _vp, _vp, _vp]),
    "smc_set_state": (_i32, [_handle, _vp, _vp, _vp, _u64]),
    "smc_get_rng_counter": (_i32, [_handle, C.POINTER(_u64)]),
    "smc_set_noise": (_i32, [_handle, _vp]),
    "smc_set_proposal_net": (_i32, [_handle, _vp, _i32, _d]),
    "smc_proposal_features": (_i32, [_handle, _d, _d, _vp]),
    "smc_nn_forward": (_i32, [_handle, _vp, _i64, _vp]),
    "smc_nn_backward": (_i32, [_handle, _vp, _i64, _vp, _vp, _vp]),
    "smc_n_params": (_i64, [_handle]),
    "smc_chunk_samples": (_i64, [_handle]),
    "smc_normalise": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "smc_systematic_resample": (_i32, [_vp, _i32, _d, _vp, _vp, _vp]),
    "smc_multinomial_resample": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "smc_philox": (_i32, [_u32, _u32, _u32, _u32, _u32, _i64, _vp, _vp]),
    "smc_proposal_targets": (_i32, [_handle, _i64, _d, C.POINTER(_d), _i32, _d, _d, _vp, _vp]),
    "smc_mlp_n_params": (_i32, [_i32]),
    "smc_mlp_forward": (_i32, [_vp, _vp, _i64, _i32, _vp, _i32, _d, _i32, _vp]),
    "smc_mlp_grad": (_i32, [_vp, _vp, _vp, _i64, _i32, _vp, C.POINTER(_d), _vp]),
    "smc_mlp_train": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32, _d, C.POINTER(_d), _vp]),
    "smc_set_proposal": (_i32, [_handle, _i32]),
    "smc_mlp_train_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32, _d, _vp, _vp]),
    "smc_profile": (_i32, [_handle, _i32]),
    "smc_profile_read": (_i32, [_handle, C.POINTER(_d), C.POINTER(_i64), C.POINTER(_d), C.POINTER(_d)]),
}

SMC_K_NAMES = ("gemm_fwd1", "gemm_dw1", "gemm_other", "head", "move", "weight", "resample", "other")
SMC_K_COUNT = len(SMC_K_NAMES)

EXPORTED = tuple(_SIGS)

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(st: int, where: str) -> None:
    if st != 0:
        raise SMCError(st, where, lib.smc_last_error().decode(errors="replace"))


def _opt(p):
    return None if p is None else C.c_void_p(int(p))


# ---------------------------------------------------------------- same names as the C ABI
def smc_status_string(status: int) -> str:
    return lib.smc_status_string(status).decode()


def smc_last_error() -> str:
    return lib.smc_last_error().decode(errors="replace")


def smc_init(cfg: smc_config, x_dev, y_dev, n_data: int, theta0_dev, m0: int, lambda0: float, stream) -> int:
    h = _handle()
    _check(lib.smc_init(C.byref(cfg), _opt(x_dev), _opt(y_dev), n_data, _opt(theta0_dev), m0, lambda0,
                        _opt(stream), C.byref(h)), "smc_init")
    return h.value


def smc_destroy(h) -> None:
    lib.smc_destroy(h)


def smc_step(h, m_k: int, lambda_k: float, want_info: bool = True):
    info = smc_step_info()
    _check(lib.smc_step(h, m_k, lambda_k, C.byref(info) if want_info else None), "smc_step")
    return info if want_info else None


def smc_step_tempered(h, m_k: int, m_split: int, lambda_a: float, lambda_b: float, want_info: bool = True):
    info = smc_step_info()
    _check(lib.smc_step_tempered(h, m_k, m_split, lambda_a, lambda_b, C.byref(info) if want_info else None),
           "smc_step_tempered")
    return info if want_info else None


def smc_segment_moments(h):
    """(E[Omega^], Var(Omega^), E[Omega], Cov(Omega, Omega^))."""
    out = (C.c_double * 4)()
    _check(lib.smc_segment_moments(h, out), "smc_segment_moments")
    return tuple(out)


def smc_resample(h, mode: int, u=None, want_result: bool = False, want_ancestors: bool = False, J: int = 0):
    uu = C.c_double(u) if u is not None else None
    res = C.c_int32(0)
    anc = (C.c_int32 * J)() if want_ancestors else None
    _check(lib.smc_resample(h, mode, C.byref(uu) if uu is not None else None,
                            C.byref(res) if want_result else None, anc), "smc_resample")
    return (bool(res.value) if want_result else None), (list(anc) if want_ancestors else None)


def smc_resample_multinomial(h, mode: int, u_dev=None, want_result: bool = False, want_ancestors: bool = False,
                             J: int = 0):
    res = C.c_int32(0)
    anc = (C.c_int32 * J)() if want_ancestors else None
    _check(lib.smc_resample_multinomial(h, mode, _opt(u_dev), C.byref(res) if want_result else None, anc),
           "smc_resample_multinomial")
    return (bool(res.value) if want_result else None), (list(anc) if want_ancestors else None)


def smc_posterior_predict(h, x_dev, y_dev, n: int, probs_dev=None, want_metrics: bool = True):
    acc, mlp = C.c_double(0.0), C.c_double(0.0)
    _check(lib.smc_posterior_predict(h, _opt(x_dev), _opt(y_dev), n, _opt(probs_dev),
                                     C.byref(acc) if want_metrics else None,
                                     C.byref(mlp) if want_metrics else None), "smc_posterior_predict")
    return (acc.value, mlp.value) if want_metrics else (None, None)


def smc_posterior_mean(h, mean_dev) -> None:
    _check(lib.smc_posterior_mean(h, _opt(mean_dev)), "smc_posterior_mean")


def smc_posterior_mean_change(h) -> float:
    r = C.c_double(0.0)
    _check(lib.smc_posterior_mean_change(h, C.byref(r)), "smc_posterior_mean_change")
    return r.value


def smc_get_state(h, theta_dev=None, logw_dev=None, loglik_dev=None, logpi_dev=None, grad_dev=None) -> None:
    _check(lib.smc_get_state(h, _opt(theta_dev), _opt(logw_dev), _opt(loglik_dev), _opt(logpi_dev),
                             _opt(grad_dev)), "smc_get_state")


def smc_set_state(h, theta_dev, logw_dev=None, logpi_dev=None, rng_counter: int = 0) -> None:
    _check(lib.smc_set_state(h, _opt(theta_dev), _opt(logw_dev), _opt(logpi_dev), rng_counter), "smc_set_state")


def smc_get_rng_counter(h) -> int:
    c = C.c_uint64(0)
    _check(lib.smc_get_rng_counter(h, C.byref(c)), "smc_get_rng_counter")
    return c.value


def smc_set_noise(h, momenta_dev) -> None:
    _check(lib.smc_set_noise(h, _opt(momenta_dev)), "smc_set_noise")


def smc_set_proposal_net(h, params_dev, n_params: int, h0: float) -> None:
    _check(lib.smc_set_proposal_net(h, _opt(params_dev), n_params, h0), "smc_set_proposal_net")


def smc_proposal_features(h, k_over_K: float, m_over_N: float, feat_dev) -> None:
    _check(lib.smc_proposal_features(h, k_over_K, m_over_N, _opt(feat_dev)), "smc_proposal_features")


def smc_nn_forward(h, theta_dev, m: int, ll_dev) -> None:
    _check(lib.smc_nn_forward(h, _opt(theta_dev), m, _opt(ll_dev)), "smc_nn_forward")


def smc_nn_backward(h, theta_dev, m: int, scale_dev, ll_dev, grad_dev) -> None:
    _check(lib.smc_nn_backward(h, _opt(theta_dev), m, _opt(scale_dev), _opt(ll_dev), _opt(grad_dev)),
           "smc_nn_backward")


def smc_n_params(h) -> int:
    return lib.smc_n_params(h)


def smc_chunk_samples(h) -> int:
    return lib.smc_chunk_samples(h)


def smc_normalise(logw_dev, J: int, logw_out_dev, stats_dev, stream) -> None:
    _check(lib.smc_normalise(_opt(logw_dev), J, _opt(logw_out_dev), _opt(stats_dev), _opt(stream)), "smc_normalise")


def smc_multinomial_resample(w_dev, J: int, u_dev, ancestors_dev, placement_dev, stream) -> None:
    _check(lib.smc_multinomial_resample(_opt(w_dev), J, _opt(u_dev), _opt(ancestors_dev), _opt(placement_dev),
                                        _opt(stream)), "smc_multinomial_resample")


def smc_systematic_resample(w_dev, J: int, u: float, ancestors_dev, placement_dev, stream) -> None:
    _check(lib.smc_systematic_resample(_opt(w_dev), J, u, _opt(ancestors_dev), _opt(placement_dev), _opt(stream)),
           "smc_systematic_resample")


def smc_philox(key0: int, key1: int, c1: int, c2: int, c3: int, n_blocks: int, out_dev, stream) -> None:
    _check(lib.smc_philox(key0, key1, c1, c2, c3, n_blocks, _opt(out_dev), _opt(stream)), "smc_philox")


def smc_profile(h, enable: bool) -> None:
    _check(lib.smc_profile(h, 1 if enable else 0), "smc_profile")


def smc_profile_read(h) -> dict:
    """{class name: (total_ms, launches, algorithmic flops, algorithmic bytes)}"""
    t = (C.c_double * SMC_K_COUNT)()
    n = (C.c_int64 * SMC_K_COUNT)()
    f = (C.c_double * SMC_K_COUNT)()
    b = (C.c_double * SMC_K_COUNT)()
    _check(lib.smc_profile_read(h, t, n, f, b), "smc_profile_read")
    return {SMC_K_NAMES[k]: (t[k], n[k], f[k], b[k]) for k in range(SMC_K_COUNT)}


def smc_proposal_targets(h, m_k: int, lambda_k: float, h_grid, k_over_K: float, accept_power: float, feat_dev,
                         target_dev) -> None:
    arr = (C.c_double * len(h_grid))(*[float(x) for x in h_grid])
    _check(lib.smc_proposal_targets(h, m_k, lambda_k, arr, len(h_grid), k_over_K, accept_power, _opt(feat_dev),
                                    _opt(target_dev)), "smc_proposal_targets")


def smc_mlp_n_params(n_groups: int) -> int:
    return lib.smc_mlp_n_params(n_groups)


def smc_mlp_forward(params_dev, feat_dev, R: int, n_groups: int, out_dev, mode: int, h0: float, bf16: bool,
                    stream) -> None:
    _check(lib.smc_mlp_forward(_opt(params_dev), _opt(feat_dev), R, n_groups, _opt(out_dev), mode, h0,
                               1 if bf16 else 0, _opt(stream)), "smc_mlp_forward")


def smc_mlp_grad(params_dev, feat_dev, target_dev, R: int, n_groups: int, grad_dev, stream) -> float:
    loss = C.c_double(0.0)
    _check(lib.smc_mlp_grad(_opt(params_dev), _opt(feat_dev), _opt(target_dev), R, n_groups, _opt(grad_dev),
                            C.byref(loss), _opt(stream)), "smc_mlp_grad")
    return loss.value


def smc_mlp_train(params_dev, adam_dev, feat_dev, target_dev, R: int, n_groups: int, first_step: int, n_steps: int,
                  lr: float, stream) -> float:
    loss = C.c_double(0.0)
    _check(lib.smc_mlp_train(_opt(params_dev), _opt(adam_dev), _opt(feat_dev), _opt(target_dev), R, n_groups,
                             first_step, n_steps, lr, C.byref(loss), _opt(stream)), "smc_mlp_train")
    return loss.value


def smc_mlp_train_noalloc(params_dev, adam_dev, feat_dev, target_dev, R: int, n_groups: int, first_step: int,
                          n_steps: int, lr: float, loss_dev, stream) -> None:
    _check(lib.smc_mlp_train_noalloc(_opt(params_dev), _opt(adam_dev), _opt(feat_dev), _opt(target_dev), R,
                                     n_groups, first_step, n_steps, lr, _opt(loss_dev), _opt(stream)),
           "smc_mlp_train_noalloc")


def smc_set_proposal(h, proposal: int) -> None:
    _check(lib.smc_set_proposal(h, proposal), "smc_set_proposal")
