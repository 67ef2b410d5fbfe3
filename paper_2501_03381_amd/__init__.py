"""MI355X-native evaluator of Gaussian-copula higher-order-interaction measures
(TC, DTC, O-information, S-information) over batches of n-plets (THOI, arXiv 2501.03381).

The compute path is the C-ABI library ``libthoi.so`` (hand-written HIP kernels for
gfx950); ``binding`` marshals arguments to it through ctypes and ``api`` exposes the
torch-facing calls.  Importing this package does not load the library; the first
call into ``api`` does, and fails loudly if it is not built.
"""
__all__ = ["api", "binding", "synth"]
