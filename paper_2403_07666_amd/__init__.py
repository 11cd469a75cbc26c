"""MI355X (gfx950) coil quench hot path: HIP kernels behind a C ABI
(include/coil.h), with a thin ctypes binding.

    from paper_2403_07666_amd import Coil
    c = Coil(workload, inputs)      # workload: coil_synth.Workload
    c.run(100)
    B = c.get(F_BZ)
"""
from .coil import (  # noqa: F401
    FP64, MIXED, ALGO_AUTO, ALGO_DIRECT, ALGO_TRANSLATION, ALGO_FFT, F_I, F_J, F_BR, F_BZ, F_T, F_PHI, F_QW, F_UW, F_E, F_EP, F_U, F_Q, F_PSI, F_R, F_Z,
    F_DI, F_JC, F_ONSET, F_QUENCH, F_Q_ONSET, F_Q_QUENCH, F_T_QUENCH, F_P_QUENCH, F_IH, F_EM_SUBSTEPS, PER_WIRE,
    AXISYMMETRIC, PLANAR, COUPLE_TRANSPORT, COUPLE_FULL, HEAT_EXPLICIT, HEAT_ADI,
    Coil, CoilError, host_ellip, lib, query, EXPORTS, FIELD_AT_SCRATCH_BYTES,
)
