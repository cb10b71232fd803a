"""MI355X-native batched evaluation and training of the OpenMP Advisor cost
model (arXiv 2301.03636): featurize -> MLP -> per-kernel argmin, plus its
training step, behind the C ABI of libadvisor.so (include/advisor.h)."""
from . import _lib
from ._lib import (AdvisorError, PRECISIONS, advisor_featurize, advisor_model_create,  # noqa: F401
                   advisor_model_destroy, advisor_model_get_adam, advisor_model_get_params,
                   advisor_model_param_count, advisor_model_set_adam, advisor_model_set_params,
                   advisor_model_set_zscore, advisor_mfma_peak, advisor_predict, advisor_profile_enable,
                   advisor_profile_read, advisor_profile_read_each, advisor_rank, advisor_rank_preds, advisor_rank_refined,
                   advisor_rank_cascade, advisor_rank_cascade_noalloc,
                   advisor_zscore_fit, last_error, advisor_mlp_saved_bytes, advisor_mlp_forward,
                   advisor_mlp_backward, advisor_train_step, advisor_model_load_params,
                   advisor_model_grads, advisor_model_calibrate_fp8, advisor_model_get_fp8_scales,
                   advisor_rank_plan_create, advisor_train_plan_create, advisor_plan_launch,
                   advisor_plan_destroy, advisor_autotune, advisor_model_set_tile_variant,
                   advisor_model_get_tile_variant, advisor_validate_offsets, advisor_topn_preds,
                   advisor_rank_topn, advisor_train_step_rmsprop, advisor_step_lr,
                   advisor_count_variants, advisor_enumerate_variants, advisor_lower_variants, advisor_classify_maps,
                   advisor_rank_multi, advisor_train_plan_create_rmsprop,
                   advisor_train_plan_create_rmsprop_multi)
from .model import Model, Plan  # noqa: F401
from .train import MLPFunction, RMSpropTrainer, Trainer, mlp, step_lr  # noqa: F401
