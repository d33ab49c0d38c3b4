"""The build's register-boundary check (CPU only): a 64-bit VALU instruction
whose 32-bit VGPR operand is the last register of the wavefront's VGPR
allocation is refused; the same instruction below the last register passes."""
from paper_2208_09985_amd.build import register_boundary_problems


def asm(next_free: int, shift_reg: int, op: str = "v_lshrrev_b64") -> str:
    return (f"_Zk:                                    ; @_Zk\n"
            f"\tv_add_u32_e32 v{shift_reg}, 1, v4\n"
            f"\t{op} v[6:7], v{shift_reg}, v[8:9]\n"
            f"\ts_endpgm\n"
            f"\t.amdhsa_kernel _Zk\n"
            f"\t\t.amdhsa_next_free_vgpr {next_free}\n"
            f"\t.end_amdhsa_kernel\n")


def test_last_register_as_shift_amount_is_refused():
    # 184 VGPRs allocated: v183 is the last one
    assert len(register_boundary_problems(asm(184, 183))) == 1
    assert len(register_boundary_problems(asm(160, 159, "v_lshlrev_b64"))) == 1


def test_register_below_the_end_of_the_allocation_passes():
    assert register_boundary_problems(asm(183, 182)) == []   # allocation rounds up to 184
    assert register_boundary_problems(asm(185, 183)) == []   # allocation 192
    assert register_boundary_problems(asm(184, 100)) == []


def test_32_bit_instructions_are_not_flagged():
    a = asm(184, 183).replace("v_lshrrev_b64 v[6:7], v183, v[8:9]", "v_lshrrev_b32_e32 v6, v183, v8")
    assert register_boundary_problems(a) == []
