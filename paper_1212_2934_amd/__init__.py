"""Barnes-Hut dipolar field and ferrofluid MD for AMD MI355X (gfx950).

The compute path is the HIP library ``libffbh.so`` behind the C ABI declared in ``include/ffbh.h``;
``binding`` marshals torch device tensors and streams into it.  Importing the package loads nothing:
the library is opened on first use and a missing library is an error, never a fallback.
"""
__all__ = ["binding", "workloads"]
