/*
 * tdes_probe.h - microbenchmarks for the hardware ceilings the 3DES kernels
 * are reported against (not part of the cipher).
 *
 * The bitsliced kernel is bound by issue of 32-bit vector ALU instructions:
 * its rounds are v_bitop3_b32 gates and key XORs with vector operands, its
 * transposes byte permutes, shifts and selects.  A gfx950 SIMD issues a
 * wave64 VALU instruction over four cycles and may issue a second one from
 * another wave in the same four cycles, for some opcodes only; these probes
 * measure the sustained lane-operation rate per opcode (rocprofv3 counters
 * SQ_INSTS_VALU / SQ_ACTIVE_INST_VALU2 give the pairing directly), the LDS
 * read rate (the table kernel's other ceiling; SQ_LDS_BANK_CONFLICT shows
 * the conflicts of each pattern), and the HBM bandwidth of a plain copy (also the reference kernel whose memory
 * counters calibrate the cipher's measured HBM traffic).
 *
 * Same conventions as tdes.h: device pointers owned by the caller, work
 * enqueued on `stream` (a hipStream_t, NULL = default), return 0 on success,
 * -1 on a bad argument (nothing enqueued), -6 if the launch failed.
 */
#ifndef TDES_PROBE_H
#define TDES_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TDES_PROBE_BITOP3 = 0,    /* v_bitop3_b32, three vector operands        */
    TDES_PROBE_XOR = 1,       /* v_xor_b32, two vector operands             */
    TDES_PROBE_XOR_SGPR = 2,  /* v_xor_b32 with one scalar operand          */
    TDES_PROBE_PERM = 3,      /* v_perm_b32 (byte permute), vector operands */
    TDES_PROBE_BFI = 4,       /* v_bfi_b32 (bit-field insert)               */
    TDES_PROBE_LSHL = 5,      /* v_lshlrev_b32 by an inline constant        */
    TDES_PROBE_LSHR = 6,      /* v_lshrrev_b32 by an inline constant        */
    TDES_PROBE_ADD = 7,       /* v_add_u32, two vector operands             */
    TDES_PROBE_BFE = 8        /* v_bfe_i32 (sign-extended bit-field extract) */
};

/* Launch `blocks` workgroups of 256 threads; every thread issues
 * 16 * iters instructions of kind `op`, then writes one word to
 * d_sink[block * 256 + thread] (d_sink holds blocks * 256 uint32).
 * Lane operations performed: blocks * 256 * 16 * iters. */
int tdes_probe_valu(int op, uint32_t *d_sink, unsigned blocks, unsigned iters, void *stream);

/* LDS read patterns for tdes_probe_lds. */
enum {
    TDES_PROBE_LDS_CONSEC = 0,   /* ds_read_b32, a wave's lanes on 64 consecutive words */
    TDES_PROBE_LDS_SAMEBANK = 1, /* ds_read_b32, all lanes of a read in one bank        */
    TDES_PROBE_LDS_BCAST = 2,    /* ds_read_b32, all lanes on one word (broadcast)      */
    TDES_PROBE_LDS_B128 = 3      /* ds_read_b128, 64 consecutive 16-byte pieces          */
};

/* Launch `blocks` workgroups of 256 threads, each with a 64 KiB LDS table;
 * every thread issues 16 * iters LDS reads of pattern `mode`, then writes
 * one word to d_sink[block * 256 + thread] (d_sink holds blocks * 256
 * uint32).  Bytes read from LDS: blocks * 256 * 16 * iters * 4 (16 for
 * TDES_PROBE_LDS_B128). */
int tdes_probe_lds(int mode, uint32_t *d_sink, unsigned blocks, unsigned iters, void *stream);

/* Copy nbytes (multiple of 16; both pointers 16-byte aligned; buffers
 * must not overlap) from d_in to d_out with 16-byte vector loads/stores. */
int tdes_probe_copy(const void *d_in, void *d_out, size_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TDES_PROBE_H */
