"""MI355X-native ddLPB: energy, adjoint solve and analytical forces of the
domain-decomposition linearised Poisson--Boltzmann model, computed by the HIP
kernels of libddlpb.so (C ABI in include/ddlpb.h)."""
from ._lib import Context, DDLPBError, load  # noqa: F401

__all__ = ["Context", "DDLPBError", "load"]
