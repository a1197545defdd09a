"""C-ABI checks that need no GPU: the library loads and exports every entry
point that include/llama.h declares; the header and the binding agree."""
import os
import re

import pytest

from paper_2102_01887_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llama.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(llama_[a-z_]+)\s*\(", text)))


def test_header_declares_the_paper_boundary():
    names = declared_functions()
    for required in ("llama_set_dag", "llama_set_profiles", "llama_targets", "llama_select"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = binding.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(binding.EXPORTS) == declared_functions()


def test_library_has_gfx950_code():
    with open(binding.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"gfx950" in blob


def test_no_gpu_means_a_loud_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(binding.LlamaError):
        binding.Llama(0)
