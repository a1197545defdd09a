"""MI355X-native per-invocation decision engine for Llama (arXiv 2102.01887).

For each pending operation invocation of a pipeline DAG it computes the
per-backend latency target (Alg. 1) and the cheapest configuration predicted
to meet it (Eq. 1), in HIP kernels for gfx950 behind the C ABI declared in
``include/llama.h``.  ``binding`` is a thin ctypes layer over that ABI;
``workloads`` draws seeded synthetic inputs.
"""
__all__ = ["binding", "workloads"]
