"""MI355X-native time propagation of the TDSE over a field-free |n,l> basis.

Method: O Broin & Nikolopoulos, arXiv:1201.6062 (Sec. 3-4, appendix B).
The compute path is the HIP library libtdse.so (C ABI in include/tdse.h);
`api` holds the thin torch-facing binding, `workloads` the seeded synthetic
inputs. Import of the binding is lazy so the input generator can be used
without loading the GPU runtime.
"""
__all__ = ["Plan", "Group", "Propagate", "piecewise_field", "ionization_yield", "tune", "TdseError", "workloads"]


def __getattr__(name):
    if name in ("Plan", "Group", "Propagate", "piecewise_field", "ionization_yield", "tune", "TdseError", "METHODS"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
