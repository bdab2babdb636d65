"""MI355X-native certified-split lexer (gfx950 HIP kernels behind a small C ABI).

The binding is argument marshalling only: every step of a scan runs in the HIP library
``liblexgpu.so`` (built in-tree by ``paper_2608_03473_amd.build``).  PyTorch provides device
memory and streams.  Importing the package does not touch the GPU; the library is loaded
on first use and its absence is an error (there is no CPU fallback).

    lx = Lexer.compile(defs)                 # defs: [(pattern, priority, discard), ...]
    r = lx.run(u8_cuda_tensor, mode=LEX_MODE_EXACT)   # r.kinds, r.lens, r.ntokens, r.error_offset
    fx = Lexer.compile_framed(defs, 0x1E)    # the set framed by a reserved byte (Section 7.1)
    b = Batch([(lx, LEX_MODE_EXACT), ...])   # many documents in one launch sequence

Also here: ``serve`` (the serving loop over batches) and ``applicability`` (certified and
useful bytes of a token set, per mode).
"""
from .abi import (LEX_EDEVICE, LEX_EINVAL, LEX_ELIMIT, LEX_EMIT_DEFAULT, LEX_EMIT_LANE,  # noqa: F401
                  LEX_ENOMEM, LEX_EOVERFLOW, LEX_ESYNTAX, LEX_MODE_DISCARD, LEX_MODE_EXACT,
                  LEX_MODE_SERIAL, LEX_OK, LexError, RunOpts, lib, lib_path)
from .lexer import DOC_DTYPE, DOC_RESULT_DTYPE, Batch, BatchResult, Lexer, RunResult  # noqa: F401

__all__ = ["Lexer", "RunResult", "Batch", "BatchResult", "DOC_DTYPE", "DOC_RESULT_DTYPE", "RunOpts",
           "LexError", "lib", "lib_path",
           "LEX_MODE_EXACT", "LEX_MODE_DISCARD", "LEX_MODE_SERIAL"]
