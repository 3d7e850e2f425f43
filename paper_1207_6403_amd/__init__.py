"""MI355X (gfx950) library for the per-timestep loop of the NMAGIC made-to-measure
particle method: hand-written HIP kernels behind the C ABI of include/m2m.h, and a
thin ctypes binding with the same entry-point names (``binding``)."""
from .binding import (M2MError, anisotropy, m2m_abi_version, m2m_autotune, m2m_create, m2m_delta_chi2, m2m_destroy,  # noqa: F401
                      m2m_get_launch, m2m_history, m2m_kernel_time, m2m_last_error, m2m_mlp_loss_grad, m2m_mlp_loss_grad_noalloc,
                      m2m_mlp_state,
                      m2m_multipole_tables,
                      m2m_observables, m2m_particles, m2m_priors, m2m_set_launch, m2m_set_tracers, m2m_shell_moments, m2m_step, m2m_step_index, m2m_tags, m2m_tracer_state,
                      m2m_weights)
