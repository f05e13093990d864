"""Two-component D3Q19 Shan-Chen lattice Boltzmann on AMD Instinct MI355X.

The computation lives in liblb.so (HIP kernels for gfx950 behind the C ABI
of include/lb.h); ``lb`` is its ctypes binding.
"""

from .lb import (  # noqa: F401
    LB_EDEVICE, LB_EINVAL, LB_KERNEL_AUTO, LB_KERNEL_FUSED, LB_KERNEL_TWO_PASS, LB_ENOMEM, LB_ENONFINITE, LB_ESTATE, LB_F16_SHIFTED, LB_F32, LB_F64, LB_OK,
    Lattice, LBError, LBLibraryMissing, LIB_PATH, SYMBOLS, library, lb_abi_version, lb_create, lb_destroy,
    lb_adjoint_begin, lb_adjoint_lambda, lb_adjoint_result, lb_adjoint_step, lb_adjoint_step_record, lb_device_bytes,
    lb_record_bytes, lb_step_record,
    lb_get_populations, lb_restore_state, lb_save_state, lb_set_coupling, lb_set_model, LB_MODEL_SHAN_CHEN, LB_MODEL_COLOUR_GRADIENT, lb_state_bytes, lb_step_between, lb_moments, lb_params, lb_params_default, lb_set_fields,
    lb_set_kernel, lb_set_populations, lb_set_stream, lb_step, lb_strerror, lb_timing, lb_timing_name, lb_timing_read,
    lb_timing_slots, lb_totals, lb_snapshot_totals,
    SingleFluid, lb1_create, lb1_destroy, lb1_get_populations, lb1_moments, lb1_set_fields, lb1_set_stream, lb1_step,
    lb1_totals, lb1_set_particles, lb1_get_particles, lb_set_particles, lb_get_particles,
)
